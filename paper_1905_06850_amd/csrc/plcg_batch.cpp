// Host side of batched and served solves: slots, HBM arena, schedule, ticks.
//
// Admission: a system needs (2l + R + 1) work vectors (FP32-refined: 2l + R + 2
// FP32 vectors, the last one the correction) plus its scaled operator
// (edge weights and D^{-1/2}); it is admitted when a slot and a first-fit block
// of the arena are free.  The coefficients are scaled here, on the host, as part
// of the operator setup: d_p = sum of the edges incident to p, s_pq = c_pq /
// sqrt(d_p d_q).  The schedule lists, for every admitted slot, one owner
// workgroup and the slot's streaming workgroups; it is rebuilt when slots come
// or go and uploaded on the stream, so launches already enqueued keep theirs.
#include "plcg_internal.h"

#include "../../include/plcg.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

using namespace plcg;

namespace {

#define BHIP(call)                                                                    \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return set_last_error(PLCG_E_HIP, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
  } while (0)

constexpr size_t kAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Block {
  size_t off, size;
};

}  // namespace

struct plcg_batch {
  plcg_batch_config cfg{};
  int l = 2, R = 2, device = 0;
  bool mixed = false;                   // FP32-refined: work vectors stored in FP32
  double inner_tol = 1e-3;
  double sigma[kLMax] = {0};
  // chunks per streaming workgroup, by the size class of a system (chunks of 512
  // unknowns: <= kSmallChunks, <= kMediumChunks, more)
  int cpb[3] = {4, 4, 4};
  // device
  char *arena = nullptr;
  size_t arena_size = 0;
  SlotDesc *d_slots = nullptr;
  BatchState *d_state = nullptr;
  double *d_part = nullptr;
  int2 *d_sched = nullptr;
  uint64_t *d_tickets = nullptr;
  SlotReport *reports = nullptr;        // mapped pinned host memory
  SlotReport *d_reports = nullptr;
  size_t sched_cap = 0;
  // host mirrors
  std::vector<SlotDesc> slots;
  std::vector<int> in_use;              // 1 while a system occupies the slot
  std::vector<uint64_t> tickets;
  std::vector<Block> slot_mem;
  std::vector<Block> free_list;         // sorted by offset
  std::map<uint64_t, int> ticket_slot;
  uint64_t next_ticket = 1;
  std::vector<int2> sched;
  bool dirty = true;
  int hint = 0;                         // streaming cache hints of the current schedule
  std::vector<int> pending_desc;        // admitted slots whose descriptors are not uploaded yet
  std::vector<BatchState> pending_state;
  std::vector<uint64_t> pending_ticket;
  int64_t tick = 0;
  // graph of a group of ticks for the current schedule
  hipGraphExec_t gexec = nullptr;
  int graph_ticks = 0;
  // registered operators (scaled once, shared by the requests that name them)
  struct Op {
    int kind, nx, ny, nz;
    int64_t n;
    double *mem;
    const double *sx, *sy, *sz, *dis;
  };
  std::vector<Op> ops;
};

namespace {

int32_t flush_admissions(plcg_batch *b, hipStream_t st);

void free_graph(plcg_batch *b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->graph_ticks = 0;
}

bool arena_alloc(plcg_batch *b, size_t size, size_t *off) {
  for (size_t k = 0; k < b->free_list.size(); ++k) {
    Block &f = b->free_list[k];
    if (f.size >= size) {
      *off = f.off;
      f.off += size;
      f.size -= size;
      if (f.size == 0) b->free_list.erase(b->free_list.begin() + k);
      return true;
    }
  }
  return false;
}

void arena_free(plcg_batch *b, Block blk) {
  auto it = std::lower_bound(b->free_list.begin(), b->free_list.end(), blk.off,
                             [](const Block &x, size_t off) { return x.off < off; });
  it = b->free_list.insert(it, blk);
  // merge with neighbours
  size_t k = it - b->free_list.begin();
  if (k + 1 < b->free_list.size() && b->free_list[k].off + b->free_list[k].size == b->free_list[k + 1].off) {
    b->free_list[k].size += b->free_list[k + 1].size;
    b->free_list.erase(b->free_list.begin() + k + 1);
  }
  if (k > 0 && b->free_list[k - 1].off + b->free_list[k - 1].size == b->free_list[k].off) {
    b->free_list[k - 1].size += b->free_list[k].size;
    b->free_list.erase(b->free_list.begin() + k);
  }
}

struct Layout {
  int64_t n;
  size_t vstride;      // elements of the storage type between work vectors
  size_t vec_bytes;    // all work vectors
  size_t x_bytes;      // an internal FP64 iterate (requests without a caller x)
  size_t nsx, nsy, nsz, bytes, op_bytes;
};

// Work vectors per system: bases 2l, ring R, p (and the FP32 correction).
int work_vectors(const plcg_batch *b) { return 2 * b->l + b->R + 1 + (b->mixed ? 1 : 0); }
size_t word_bytes(const plcg_batch *b) { return b->mixed ? 4 : 8; }

int32_t layout(const plcg_batch *b, const plcg_system_desc *sys, Layout *L) {
  if (sys == nullptr) return PLCG_E_INVALID;
  if (sys->kind != PLCG_OP_STENCIL2D5 && sys->kind != PLCG_OP_STENCIL3D7) return PLCG_E_INVALID;
  const bool d3 = sys->kind == PLCG_OP_STENCIL3D7;
  const int64_t nx = sys->nx, ny = sys->ny, nz = d3 ? sys->nz : 1;
  if (nx < 1 || ny < 1 || nz < 1 || (!d3 && sys->nz > 1)) return PLCG_E_INVALID;
  L->n = nx * ny * nz;
  if (L->n > kMaxUnknowns) return PLCG_E_INVALID;
  const size_t w = word_bytes(b);
  L->vstride = round_up((size_t)L->n * w, kAlign) / w;
  L->vec_bytes = (size_t)work_vectors(b) * L->vstride * w;
  L->x_bytes = round_up((size_t)L->n * 8, kAlign);
  L->nsx = (size_t)(nx + 1) * ny * nz;
  L->nsy = (size_t)nx * (ny + 1) * nz;
  L->nsz = d3 ? (size_t)nx * ny * (nz + 1) : 0;
  L->op_bytes = round_up(L->nsx * 8, kAlign) + round_up(L->nsy * 8, kAlign) +
                round_up(L->nsz * 8, kAlign) + round_up((size_t)L->n * 8, kAlign);
  L->bytes = L->vec_bytes + L->op_bytes;
  return PLCG_OK;
}

}  // namespace

// Host: the edge weights VarOp reads, from coefficient arrays in host memory
// (NULL: all 1; layouts as plcg_system_desc).  jacobi: w_pq = c_pq d_p^{-1/2}
// d_q^{-1/2} and dd = D^{-1/2}; else w_pq = c_pq and dd = d; d_p is the sum of
// the edges at p, boundary edges included.  Boundary edges get weight 0
// (VarOp never reads them).  wx, wy, wz, dd hold (nx+1) ny nz, nx (ny+1) nz,
// nx ny (nz+1) (3D) and nx ny nz values.
int32_t plcg::edge_weights(int nx, int ny, int nz, bool d3, const double *cx, const double *cy,
                           const double *cz, bool jacobi, double *wx, double *wy, double *wz,
                           double *dd) {
  const size_t nsx = (size_t)(nx + 1) * ny * nz, nsy = (size_t)nx * (ny + 1) * nz;
  const size_t nsz = d3 ? (size_t)nx * ny * (nz + 1) : 0;
  for (size_t k = 0; k < nsx; ++k) wx[k] = cx ? cx[k] : 1.0;
  for (size_t k = 0; k < nsy; ++k) wy[k] = cy ? cy[k] : 1.0;
  for (size_t k = 0; k < nsz; ++k) wz[k] = cz ? cz[k] : 1.0;
  for (size_t k = 0; k < nsx; ++k)
    if (!(std::isfinite(wx[k]) && wx[k] > 0.0))
      return set_last_error(PLCG_E_INVALID, "edge coefficients must be positive and finite");
  for (size_t k = 0; k < nsy; ++k)
    if (!(std::isfinite(wy[k]) && wy[k] > 0.0))
      return set_last_error(PLCG_E_INVALID, "edge coefficients must be positive and finite");
  for (size_t k = 0; k < nsz; ++k)
    if (!(std::isfinite(wz[k]) && wz[k] > 0.0))
      return set_last_error(PLCG_E_INVALID, "edge coefficients must be positive and finite");
  double *cxv = wx, *cyv = wy, *czv = wz;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t p = x + (int64_t)nx * (y + (int64_t)ny * z);
        const int64_t row = y + (int64_t)ny * z;
        double d = cxv[row * (nx + 1) + x] + cxv[row * (nx + 1) + x + 1] +
                   cyv[((int64_t)z * (ny + 1) + y) * nx + x] +
                   cyv[((int64_t)z * (ny + 1) + y + 1) * nx + x];
        if (d3) d += czv[p] + czv[p + (int64_t)nx * ny];
        if (!(d > 0.0) || !std::isfinite(d))
          return set_last_error(PLCG_E_INVALID, "edge coefficients must be positive and finite");
        dd[p] = jacobi ? 1.0 / std::sqrt(d) : d;
      }
  // scaling factor of unknown p: D^{-1/2} (jacobi) or 1
  auto f = [&](int64_t p) { return jacobi ? dd[p] : 1.0; };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x <= nx; ++x) {
        const int64_t row = y + (int64_t)ny * z;
        const int64_t p = x + (int64_t)nx * row;
        double &c = cxv[row * (nx + 1) + x];
        c = (x > 0 && x < nx) ? (jacobi ? c * f(p - 1) * f(p) : c) : 0.0;
      }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y <= ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double &c = cyv[((int64_t)z * (ny + 1) + y) * nx + x];
        const int64_t p = x + (int64_t)nx * (y + (int64_t)ny * z);
        c = (y > 0 && y < ny) ? (jacobi ? c * f(p - nx) * f(p) : c) : 0.0;
      }
  if (d3)
    for (int z = 0; z <= nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          double &c = czv[((int64_t)z * ny + y) * nx + x];
          const int64_t p = x + (int64_t)nx * (y + (int64_t)ny * z);
          const int64_t plane = (int64_t)nx * ny;
          c = (z > 0 && z < nz) ? (jacobi ? c * f(p - plane) * f(p) : c) : 0.0;
        }
  return PLCG_OK;
}

namespace {

// Scale the edge coefficients of `sys` (Jacobi: s_pq = c_pq / sqrt(d_p d_q), d_p = sum
// of the edges at p) and copy sx, sy, sz, D^{-1/2} to `dst` (device, L.op_bytes).
int32_t upload_operator(const plcg_system_desc *sys, const Layout &L, char *dst, hipStream_t st,
                        const double **psx, const double **psy, const double **psz,
                        const double **pdis) {
  const bool d3 = sys->kind == PLCG_OP_STENCIL3D7;
  const int nx = sys->nx, ny = sys->ny, nz = d3 ? sys->nz : 1;
  const int64_t n = L.n;
  std::vector<double> cx(L.nsx), cy(L.nsy), cz(L.nsz);
  std::vector<double> dis(n);
  const int32_t e = edge_weights(nx, ny, nz, d3, sys->cx, sys->cy, d3 ? sys->cz : nullptr, true,
                                 cx.data(), cy.data(), cz.data(), dis.data());
  if (e != PLCG_OK) return e;
  char *q = dst;
  double *sx = reinterpret_cast<double *>(q);
  q += round_up(L.nsx * 8, kAlign);
  double *sy = reinterpret_cast<double *>(q);
  q += round_up(L.nsy * 8, kAlign);
  double *sz = reinterpret_cast<double *>(q);
  q += round_up(L.nsz * 8, kAlign);
  double *ds = reinterpret_cast<double *>(q);
  BHIP(hipMemcpyAsync(sx, cx.data(), L.nsx * 8, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(sy, cy.data(), L.nsy * 8, hipMemcpyHostToDevice, st));
  if (d3) BHIP(hipMemcpyAsync(sz, cz.data(), L.nsz * 8, hipMemcpyHostToDevice, st));
  BHIP(hipMemcpyAsync(ds, dis.data(), n * 8, hipMemcpyHostToDevice, st));
  // the host vectors are temporaries: wait until the copies have read them
  BHIP(hipStreamSynchronize(st));
  *psx = sx;
  *psy = sy;
  *psz = sz;
  *pdis = ds;
  return PLCG_OK;
}

constexpr int kSmallChunks = 8, kMediumChunks = 64;
int size_class(int nchunks) { return nchunks <= kSmallChunks ? 0 : nchunks <= kMediumChunks ? 1 : 2; }

int blocks_for(const plcg_batch *b, int nchunks) {
  const int c = b->cpb[size_class(nchunks)];
  int nb = (nchunks + c - 1) / c;
  return std::max(1, std::min(nb, kMaxStream));
}

// Streaming cache hints of the sweeps (measured on 512 systems, 5 GB: non-temporal
// loads and stores +6 % solves/s): taken once what the admitted systems stream
// per tick outgrows the 256 MiB memory-side cache, where the alternating tick
// order would otherwise find it.
int batch_hint(const plcg_batch *b) {
  const size_t w = b->mixed ? 4 : 8;
  size_t bytes = 0;
  for (size_t s = 0; s < b->slots.size(); ++s) {
    if (!b->in_use[s]) continue;
    const SlotDesc &d = b->slots[s];
    bytes += (size_t)d.n * ((size_t)work_vectors(b) * w + (d.d3 ? 3 : 2) * 8 + 3 * 8);
  }
  return bytes > ((size_t)256 << 20) ? (kHintLoads | kHintStores) : 0;
}

void rebuild_schedule(plcg_batch *b) {
  b->sched.clear();
  b->hint = batch_hint(b);
  for (size_t s = 0; s < b->slots.size(); ++s) {
    if (!b->in_use[s]) continue;
    b->sched.push_back(make_int2((int)s, -1));
    for (int k = 0; k < b->slots[s].nblocks; ++k) b->sched.push_back(make_int2((int)s, k));
  }
}

int32_t upload_schedule(plcg_batch *b, hipStream_t st) {
  rebuild_schedule(b);
  if (b->sched.size() > b->sched_cap) {
    // enqueued launches may still read the old table: wait for them first
    BHIP(hipStreamSynchronize(st));
    if (b->d_sched) BHIP(hipFree(b->d_sched));
    b->sched_cap = std::max<size_t>(b->sched.size() * 2, 1024);
    BHIP(hipMalloc(reinterpret_cast<void **>(&b->d_sched), b->sched_cap * sizeof(int2)));
  }
  if (!b->sched.empty()) {
    BHIP(hipMemcpyAsync(b->d_sched, b->sched.data(), b->sched.size() * sizeof(int2),
                        hipMemcpyHostToDevice, st));
    // the host vector is rebuilt on the next change: let the copy read it first
    BHIP(hipStreamSynchronize(st));
  }
  free_graph(b);
  b->dirty = false;
  return PLCG_OK;
}

int32_t launch_ticks(plcg_batch *b, int ticks, hipStream_t st) {
  BatchArgs a;
  a.slots = b->d_slots;
  a.state = b->d_state;
  a.part = b->d_part;
  a.sched = b->d_sched;
  a.reports = b->d_reports;
  a.tickets = b->d_tickets;
  a.l = b->l;
  a.mixed = b->mixed ? 1 : 0;
  a.hint = b->hint;
  const int grid = (int)b->sched.size();
  for (int k = 0; k < ticks; ++k) {
    a.tick = (int32_t)(b->tick & 1);
    BHIP(launch_batch_tick(a, grid, st));
    ++b->tick;
  }
  return PLCG_OK;
}

constexpr int kGraphTicks = 16;   // even, so a replay starts and ends on the same parity

int32_t run_ticks(plcg_batch *b, int ticks, hipStream_t st) {
  {
    int32_t e = flush_admissions(b, st);
    if (e != PLCG_OK) return e;
  }
  if (b->dirty) {
    int32_t e = upload_schedule(b, st);
    if (e != PLCG_OK) return e;
  }
  if (b->sched.empty()) return PLCG_OK;
  if (!b->cfg.use_graph) return launch_ticks(b, ticks, st);
  // Replay whole groups from the graph; the remainder and parity fix-ups directly.
  if ((b->tick & 1) && ticks > 0) {
    int32_t e = launch_ticks(b, 1, st);
    if (e != PLCG_OK) return e;
    --ticks;
  }
  if (ticks >= kGraphTicks && b->gexec == nullptr) {
    hipStream_t cap;
    BHIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g;
    int64_t saved = b->tick;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int32_t e = he == hipSuccess ? launch_ticks(b, kGraphTicks, cap) : PLCG_E_HIP;
    hipError_t he2 = hipStreamEndCapture(cap, &g);
    b->tick = saved;
    (void)hipStreamDestroy(cap);
    if (e != PLCG_OK || he2 != hipSuccess) return set_last_error(PLCG_E_HIP, "graph capture failed");
    BHIP(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    b->graph_ticks = kGraphTicks;
  }
  while (ticks >= kGraphTicks && b->gexec) {
    BHIP(hipGraphLaunch(b->gexec, st));
    b->tick += kGraphTicks;
    ticks -= kGraphTicks;
  }
  return launch_ticks(b, ticks, st);
}

}  // namespace

extern "C" {

plcg_status plcg_batch_create(const plcg_batch_config *cfg, plcg_batch **out) {
  if (out == nullptr || cfg == nullptr) return set_last_error(PLCG_E_INVALID, "NULL argument");
  *out = nullptr;
  if (cfg->l < 2 || cfg->l > 5) return set_last_error(PLCG_E_INVALID, "batched l must be in 2..5");
  if (cfg->max_slots < 1 || cfg->max_slots > 65536)
    return set_last_error(PLCG_E_INVALID, "max_slots must be in 1..65536");
  if (cfg->arena_bytes <= 0) return set_last_error(PLCG_E_INVALID, "arena_bytes must be > 0");
  double lo = cfg->lambda_min, hi = cfg->lambda_max;
  if (lo == 0.0 && hi == 0.0) hi = 2.0;
  if (!(hi > lo)) return set_last_error(PLCG_E_INVALID, "need lambda_min < lambda_max");
  if (cfg->precision != PLCG_PREC_FP64 && cfg->precision != PLCG_PREC_FP32_REFINED)
    return set_last_error(PLCG_E_INVALID, "unknown precision");
  if (cfg->precision == PLCG_PREC_FP32_REFINED && !(cfg->inner_tol < 1.0))
    return set_last_error(PLCG_E_INVALID, "inner_tol must be < 1");
  plcg_batch *b = new plcg_batch();
  b->mixed = cfg->precision == PLCG_PREC_FP32_REFINED;
  b->inner_tol = cfg->inner_tol > 0.0 ? cfg->inner_tol : 1e-3;
  b->cfg = *cfg;
  b->cfg.lambda_min = lo;
  b->cfg.lambda_max = hi;
  if (b->cfg.max_restarts < 0) b->cfg.max_restarts = 100;
  b->l = cfg->l;
  b->R = b->l - 1 > 2 ? b->l - 1 : 2;
  for (int &c : b->cpb) c = cfg->chunks_per_block > 0 ? cfg->chunks_per_block : 4;
  // Eq. (chebyshev)
  for (int i = 0; i < b->l; ++i)
    b->sigma[i] = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos((2 * i + 1) * M_PI / (2 * b->l));
  const int S = cfg->max_slots;
  b->slots.assign(S, SlotDesc{});
  b->in_use.assign(S, 0);
  b->tickets.assign(S, 0);
  b->slot_mem.assign(S, Block{0, 0});
  b->arena_size = round_up((size_t)cfg->arena_bytes, kAlign);
  auto bad = [&](const char *what, hipError_t e) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (b->arena) (void)hipFree(b->arena);
    if (b->d_slots) (void)hipFree(b->d_slots);
    if (b->d_state) (void)hipFree(b->d_state);
    if (b->d_part) (void)hipFree(b->d_part);
    if (b->d_tickets) (void)hipFree(b->d_tickets);
    if (b->reports) (void)hipHostFree(b->reports);
    delete b;
    return set_last_error(PLCG_E_NOMEM, m.c_str());
  };
  hipError_t e;
  if ((e = hipGetDevice(&b->device)) != hipSuccess) return bad("hipGetDevice", e);
  if ((e = hipMalloc(reinterpret_cast<void **>(&b->arena), b->arena_size)) != hipSuccess)
    return bad("hipMalloc(arena)", e);
  if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_slots), sizeof(SlotDesc) * S)) != hipSuccess)
    return bad("hipMalloc(slots)", e);
  if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_state), sizeof(BatchState) * 2 * S)) !=
      hipSuccess)
    return bad("hipMalloc(state)", e);
  const size_t part_bytes = sizeof(double) * (size_t)S * 2 * (b->l + 1) * kMaxStream;
  if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_part), part_bytes)) != hipSuccess)
    return bad("hipMalloc(partials)", e);
  if ((e = hipMalloc(reinterpret_cast<void **>(&b->d_tickets), sizeof(uint64_t) * S)) != hipSuccess)
    return bad("hipMalloc(tickets)", e);
  if ((e = hipHostMalloc(reinterpret_cast<void **>(&b->reports), sizeof(SlotReport) * S,
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return bad("hipHostMalloc(reports)", e);
  std::memset(b->reports, 0, sizeof(SlotReport) * S);
  void *dp = nullptr;
  if ((e = hipHostGetDevicePointer(&dp, b->reports, 0)) != hipSuccess)
    return bad("hipHostGetDevicePointer", e);
  b->d_reports = reinterpret_cast<SlotReport *>(dp);
  if ((e = hipMemset(b->d_state, 0, sizeof(BatchState) * 2 * S)) != hipSuccess)
    return bad("hipMemset", e);
  if ((e = hipMemset(b->d_part, 0, part_bytes)) != hipSuccess) return bad("hipMemset", e);
  b->free_list.push_back(Block{0, b->arena_size});
  *out = b;
  return PLCG_OK;
}

int64_t plcg_batch_footprint(const plcg_batch *b, const plcg_system_desc *sys) {
  if (b == nullptr) return -1;
  Layout L;
  if (layout(b, sys, &L) != PLCG_OK) return -1;
  return (int64_t)L.bytes;
}

}  // extern "C"

namespace {

// Admit a system whose scaled operator is at (sx, sy, sz, dis); `own_op` extra
// bytes of the slot's arena block hold a private copy (plcg_batch_add).
int32_t admit(plcg_batch *b, const plcg_system_desc *sys, const Layout &L, bool private_op,
              const plcg_system_desc *op_src, const double *sx, const double *sy,
              const double *sz, const double *dis, const double *d_b, double *d_x, double tol,
              int32_t maxit, hipStream_t st, uint64_t *ticket) {
  int slot = -1;
  for (size_t s = 0; s < b->slots.size(); ++s)
    if (!b->in_use[s]) {
      slot = (int)s;
      break;
    }
  if (slot < 0) return set_last_error(PLCG_E_BUSY, "no free slot");
  // work vectors, then an internal FP64 x if the caller gives none, then a
  // private operator copy
  const size_t vec_bytes = L.vec_bytes + (d_x == nullptr ? L.x_bytes : 0);
  const size_t bytes = vec_bytes + (private_op ? L.op_bytes : 0);
  size_t off = 0;
  if (!arena_alloc(b, bytes, &off)) return set_last_error(PLCG_E_BUSY, "not enough arena space");
  char *base = b->arena + off;
  if (private_op) {
    int32_t e = upload_operator(op_src, L, base + vec_bytes, st, &sx, &sy, &sz, &dis);
    if (e != PLCG_OK) {
      arena_free(b, Block{off, bytes});
      return e;
    }
  }
  const bool d3 = sys->kind == PLCG_OP_STENCIL3D7;
  SlotDesc sd{};
  sd.vec = reinterpret_cast<double *>(base);
  sd.vstride = (int64_t)L.vstride;
  sd.sx = sx;
  sd.sy = sy;
  sd.sz = sz;
  sd.dis = dis;
  sd.b = d_b;
  sd.x = d_x != nullptr ? d_x : reinterpret_cast<double *>(base + L.vec_bytes);
  sd.nx = sys->nx;
  sd.ny = sys->ny;
  sd.nz = d3 ? sys->nz : 1;
  sd.d3 = d3 ? 1 : 0;
  sd.n = (int32_t)L.n;
  sd.nchunks = (int32_t)((L.n + kChunk - 1) / kChunk);
  sd.nblocks = blocks_for(b, sd.nchunks);
  sd.maxit = maxit;
  sd.max_restarts = b->cfg.max_restarts;
  sd.mixed = b->mixed ? 1 : 0;
  sd.tol = tol;
  sd.inner_tol = b->inner_tol;
  BatchState bs;
  std::memset(&bs, 0, sizeof(bs));
  bs.d.l = b->l;
  for (int k = 0; k < kLMax; ++k) bs.d.sigma[k] = b->sigma[k];
  bs.phase = kInit;
  bs.first = 1;
  BatchState pair[2] = {bs, bs};
  const uint64_t tk = b->next_ticket++;
  // Stream-ordered uploads: launches already enqueued see the slot as it was.
  if (d_x == nullptr) BHIP(hipMemsetAsync(sd.x, 0, (size_t)L.n * 8, st));
  b->slots[slot] = sd;
  b->pending_desc.push_back(slot);
  b->pending_state.push_back(pair[0]);
  b->pending_ticket.push_back(tk);
  b->reports[slot].phase = kInit;
  b->reports[slot].ticket = tk;
  b->in_use[slot] = 1;
  b->tickets[slot] = tk;
  b->slot_mem[slot] = Block{off, bytes};
  b->ticket_slot[tk] = slot;
  b->dirty = true;
  *ticket = tk;
  return PLCG_OK;
}

// Upload the descriptors and initial states of newly admitted slots (one copy
// each for all of them), ahead of the next launch.
int32_t flush_admissions(plcg_batch *b, hipStream_t st) {
  if (b->pending_desc.empty()) return PLCG_OK;
  for (size_t k = 0; k < b->pending_desc.size(); ++k) {
    const int slot = b->pending_desc[k];
    BatchState pair[2] = {b->pending_state[k], b->pending_state[k]};
    BHIP(hipMemcpyAsync(b->d_slots + slot, &b->slots[slot], sizeof(SlotDesc), hipMemcpyHostToDevice, st));
    BHIP(hipMemcpyAsync(b->d_state + 2 * slot, pair, sizeof(pair), hipMemcpyHostToDevice, st));
    BHIP(hipMemcpyAsync(b->d_tickets + slot, &b->pending_ticket[k], sizeof(uint64_t),
                        hipMemcpyHostToDevice, st));
  }
  BHIP(hipStreamSynchronize(st));
  b->pending_desc.clear();
  b->pending_state.clear();
  b->pending_ticket.clear();
  return PLCG_OK;
}

}  // namespace

int64_t plcg::batch_op_unknowns(const plcg_batch *b, int32_t op_id) {
  if (b == nullptr || op_id < 0 || op_id >= (int32_t)b->ops.size()) return -1;
  return b->ops[op_id].n;
}

extern "C" {

plcg_status plcg_batch_add(plcg_batch *b, const plcg_system_desc *sys, const double *d_b,
                           double *d_x, double tol, int32_t maxit, void *stream,
                           uint64_t *ticket) {
  if (b == nullptr || ticket == nullptr || d_b == nullptr)
    return set_last_error(PLCG_E_INVALID, "NULL argument");
  if ((reinterpret_cast<uintptr_t>(d_b) & 15) || (reinterpret_cast<uintptr_t>(d_x) & 15))
    return set_last_error(PLCG_E_INVALID, "vectors must be 16-byte aligned");
  if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 0)
    return set_last_error(PLCG_E_INVALID, "need tol > 0 and maxit >= 0");
  Layout L;
  if (layout(b, sys, &L) != PLCG_OK) return set_last_error(PLCG_E_INVALID, "bad system descriptor");
  return admit(b, sys, L, true, sys, nullptr, nullptr, nullptr, nullptr, d_b, d_x, tol, maxit,
               reinterpret_cast<hipStream_t>(stream), ticket);
}

plcg_status plcg_batch_register(plcg_batch *b, const plcg_system_desc *sys, void *stream,
                                int32_t *op_id) {
  if (b == nullptr || sys == nullptr || op_id == nullptr)
    return set_last_error(PLCG_E_INVALID, "NULL argument");
  Layout L;
  if (layout(b, sys, &L) != PLCG_OK) return set_last_error(PLCG_E_INVALID, "bad system descriptor");
  BHIP(hipSetDevice(b->device));
  plcg_batch::Op op{};
  op.kind = sys->kind;
  op.nx = sys->nx;
  op.ny = sys->ny;
  op.nz = sys->kind == PLCG_OP_STENCIL3D7 ? sys->nz : 1;
  op.n = L.n;
  hipError_t he = hipMalloc(reinterpret_cast<void **>(&op.mem), L.op_bytes);
  if (he != hipSuccess)
    return set_last_error(PLCG_E_NOMEM, (std::string("hipMalloc(operator): ") + hipGetErrorString(he)).c_str());
  int32_t e = upload_operator(sys, L, reinterpret_cast<char *>(op.mem),
                              reinterpret_cast<hipStream_t>(stream), &op.sx, &op.sy, &op.sz, &op.dis);
  if (e != PLCG_OK) {
    (void)hipFree(op.mem);
    return e;
  }
  b->ops.push_back(op);
  *op_id = (int32_t)b->ops.size() - 1;
  return PLCG_OK;
}

int64_t plcg_batch_request_footprint(const plcg_batch *b, int32_t op_id, int32_t internal_x) {
  if (b == nullptr || op_id < 0 || op_id >= (int32_t)b->ops.size()) return -1;
  const size_t n = (size_t)b->ops[op_id].n;
  const size_t w = word_bytes(b);
  return (int64_t)((size_t)work_vectors(b) * (round_up(n * w, kAlign) / w) * w +
                   (internal_x ? round_up(n * 8, kAlign) : 0));
}

plcg_status plcg_batch_add_op(plcg_batch *b, int32_t op_id, const double *d_b, double *d_x,
                              double tol, int32_t maxit, void *stream, uint64_t *ticket) {
  if (b == nullptr || ticket == nullptr || d_b == nullptr)
    return set_last_error(PLCG_E_INVALID, "NULL argument");
  if (op_id < 0 || op_id >= (int32_t)b->ops.size())
    return set_last_error(PLCG_E_INVALID, "unknown operator");
  if ((reinterpret_cast<uintptr_t>(d_b) & 15) || (reinterpret_cast<uintptr_t>(d_x) & 15))
    return set_last_error(PLCG_E_INVALID, "vectors must be 16-byte aligned");
  if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 0)
    return set_last_error(PLCG_E_INVALID, "need tol > 0 and maxit >= 0");
  const plcg_batch::Op &op = b->ops[op_id];
  plcg_system_desc sys{op.kind, op.nx, op.ny, op.nz, nullptr, nullptr, nullptr};
  Layout L;
  if (layout(b, &sys, &L) != PLCG_OK) return set_last_error(PLCG_E_INVALID, "bad operator");
  return admit(b, &sys, L, false, nullptr, op.sx, op.sy, op.sz, op.dis, d_b, d_x, tol, maxit,
               reinterpret_cast<hipStream_t>(stream), ticket);
}

plcg_status plcg_batch_step(plcg_batch *b, int32_t ticks, void *stream) {
  if (b == nullptr || ticks < 0) return set_last_error(PLCG_E_INVALID, "bad argument");
  BHIP(hipSetDevice(b->device));
  return run_ticks(b, ticks, reinterpret_cast<hipStream_t>(stream));
}

plcg_status plcg_batch_poll(plcg_batch *b, uint64_t ticket, plcg_result *out) {
  if (b == nullptr) return set_last_error(PLCG_E_INVALID, "NULL batch");
  auto it = b->ticket_slot.find(ticket);
  if (it == b->ticket_slot.end()) return set_last_error(PLCG_E_INVALID, "unknown ticket");
  const int slot = it->second;
  volatile SlotReport *rp = b->reports + slot;
  if (rp->phase != kDone || rp->ticket != ticket) return PLCG_NOT_READY;
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->iters = rp->iters;
    out->restarts = rp->restarts;
    out->reason = rp->reason;
    out->rnorm0 = rp->rnorm0;
    out->rec_relres = rp->res_scaled;
    out->true_relres = rp->res_orig;
    out->outer = rp->outer;
  }
  b->in_use[slot] = 0;
  arena_free(b, b->slot_mem[slot]);
  b->slot_mem[slot] = Block{0, 0};
  b->ticket_slot.erase(it);
  b->dirty = true;
  return PLCG_OK;
}

int32_t plcg_batch_active(const plcg_batch *b) {
  if (b == nullptr) return -1;
  return (int32_t)b->ticket_slot.size();
}

int32_t plcg_batch_grid(const plcg_batch *b) {
  if (b == nullptr) return -1;
  if (b->dirty) {
    int g = 0;
    for (size_t s = 0; s < b->slots.size(); ++s)
      if (b->in_use[s]) g += 1 + b->slots[s].nblocks;
    return g;
  }
  return (int32_t)b->sched.size();
}

int32_t plcg_batch_chunks_per_block(const plcg_batch *b) { return b ? b->cpb[2] : -1; }

plcg_status plcg_batch_set_schedule(plcg_batch *b, const int32_t *cpb) {
  if (b == nullptr || cpb == nullptr) return set_last_error(PLCG_E_INVALID, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (cpb[k] < 1 || cpb[k] > kMaxStream)
      return set_last_error(PLCG_E_INVALID, "chunks per workgroup must be in 1..1024");
  for (int k = 0; k < 3; ++k) b->cpb[k] = cpb[k];
  // systems already admitted keep their workgroups until the next autotune;
  // the choice applies to systems admitted from now on
  return PLCG_OK;
}

plcg_status plcg_batch_get_schedule(const plcg_batch *b, int32_t *cpb) {
  if (b == nullptr || cpb == nullptr) return set_last_error(PLCG_E_INVALID, "NULL argument");
  for (int k = 0; k < 3; ++k) cpb[k] = b->cpb[k];
  return PLCG_OK;
}

plcg_status plcg_batch_autotune(plcg_batch *b, int32_t ticks, void *stream) {
  if (b == nullptr || ticks < 1) return set_last_error(PLCG_E_INVALID, "bad argument");
  BHIP(hipSetDevice(b->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  {
    int32_t e = flush_admissions(b, st);
    if (e != PLCG_OK) return e;
  }
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  // New workgroup counts for every admitted system, in the table and on the device.
  auto apply = [&]() -> int32_t {
    for (size_t s = 0; s < b->slots.size(); ++s)
      if (b->in_use[s]) {
        b->slots[s].nblocks = blocks_for(b, b->slots[s].nchunks);
        BHIP(hipMemcpyAsync(b->d_slots + s, &b->slots[s], sizeof(SlotDesc), hipMemcpyHostToDevice,
                            st));
      }
    b->dirty = true;
    return PLCG_OK;
  };
  // Time `ticks` launches of the live batch under the current choice, per active
  // unknown (systems that finish between trials shrink the work of later ones).
  auto trial = [&](double *cost) -> int32_t {
    int32_t e = apply();
    if (e == PLCG_OK) e = run_ticks(b, 2, st);   // settle: the new partial count reaches the owners
    if (e != PLCG_OK) return e;
    int64_t active = 0;
    for (size_t s = 0; s < b->slots.size(); ++s)
      if (b->in_use[s] && b->reports[s].phase != kDone) active += b->slots[s].n;
    BHIP(hipEventRecord(e0, st));
    if ((e = run_ticks(b, ticks, st)) != PLCG_OK) return e;
    BHIP(hipEventRecord(e1, st));
    BHIP(hipEventSynchronize(e1));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, e0, e1));
    *cost = (double)ms / (double)std::max<int64_t>(active, 1);
    return PLCG_OK;
  };
  const int cands[] = {1, 2, 4, 8, 16};
  // 1) one size for every class; 2) each class in turn (largest first), the
  // others held at their best so far.
  int best_all = b->cpb[2];
  double best = 1e300;
  for (int c : cands) {
    for (int &k : b->cpb) k = c;
    double cost;
    int32_t e = trial(&cost);
    if (e != PLCG_OK) return e;
    if (cost < best) {
      best = cost;
      best_all = c;
    }
  }
  for (int &k : b->cpb) k = best_all;
  for (int cls = 2; cls >= 0; --cls) {
    int best_c = b->cpb[cls];
    double best_cls = 1e300;
    for (int c : cands) {
      b->cpb[cls] = c;
      double cost;
      int32_t e = trial(&cost);
      if (e != PLCG_OK) return e;
      if (cost < best_cls) {
        best_cls = cost;
        best_c = c;
      }
    }
    b->cpb[cls] = best_c;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return apply();
}

plcg_status plcg_batch_destroy(plcg_batch *b) {
  if (b == nullptr) return PLCG_OK;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_graph(b);
  for (auto &op : b->ops) (void)hipFree(op.mem);
  if (b->arena) (void)hipFree(b->arena);
  if (b->d_slots) (void)hipFree(b->d_slots);
  if (b->d_state) (void)hipFree(b->d_state);
  if (b->d_part) (void)hipFree(b->d_part);
  if (b->d_sched) (void)hipFree(b->d_sched);
  if (b->d_tickets) (void)hipFree(b->d_tickets);
  if (b->reports) (void)hipHostFree(b->reports);
  delete b;
  return PLCG_OK;
}

}  // extern "C"
