// Device helpers shared by the single-system and the batched kernels of libplcg.
#pragma once

#include <type_traits>

#include "plcg_internal.h"

#include <math.h>

namespace plcg {

// v from the lane `CTRL` selects (a DPP lane pattern), 0 in the rows that
// ROWS leaves out, and in lanes whose source lies outside the wave.  All 64
// lanes must be active.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
// v of the previous lane of the wave (wave_shr:1; 0 in lane 0) and of the next
// lane (wave_shl:1; 0 in lane 63).
__device__ inline double lane_prev(double v) { return dpp_move<0x138, 0xF>(v); }
__device__ inline double lane_next(double v) { return dpp_move<0x130, 0xF>(v); }

// ---------------------------------------------------------------------------
// Chunk scheduling
// ---------------------------------------------------------------------------

struct ChunkIter {
  int c, end, step;
  int flip;   // >= 0: positions are mirrored inside the band, at() = flip - c
  __device__ inline int at() const { return flip >= 0 ? flip - c : c; }
};

// Streaming workgroups are blockIdx.x = first .. first + nstream - 1 (first is 0
// or 1, nstream a multiple of 8); workgroup b sits on XCD b % 8 and takes band
// b % 8 of the chunks.  The workgroups of a band move through it together, so
// a sweep touches each band front to back; with rev the band is walked back to
// front.  Alternating the two from one sweep to the next starts every sweep on
// the data the previous one touched last, which is what the 256 MB memory-side
// cache still holds when a solve's vectors only just outgrow it.
__device__ inline ChunkIter xcd_chunks(int nchunks, int nstream, int first, bool rev = false) {
  const int band = blockIdx.x % kXcds;
  const int lb = (blockIdx.x - first) / kXcds;
  const int nlb = nstream / kXcds;
  const int lo = (int)(((long long)band * nchunks) / kXcds);
  const int hi = (int)(((long long)(band + 1) * nchunks) / kXcds);
  return ChunkIter{lo + lb, hi, nlb, rev ? lo + hi - 1 : -1};
}

struct Grid {
  int n, nx, ny, nz;
};

// Order in which the chunks of a 3D grid are visited.  In plain index order the
// z-neighbours of a chunk are a whole plane of chunks away, and by the time a
// plane is read again as the neighbour of the next one the XCD's L2 has long
// evicted it.  When a plane is a whole number of chunks, the chunks are visited
// by column tiles of `tile` chunks: (tile, z, chunk in tile), so the workgroups
// of an XCD, which run consecutive positions of this order side by side, read a
// tile's planes a few chunks apart.  Visiting order is all that changes.
struct ChunkOrder {
  int cpp, tile, per_tile;   // chunks per plane, chunks per tile, nz * tile; cpp == 0: identity
  __device__ inline int phys(int c) const {
    if (cpp == 0) return c;
    const int t = c / per_tile;
    const int r = c - t * per_tile;
    const int z = r / tile;
    return z * cpp + t * tile + (r - z * tile);
  }
};

__device__ inline ChunkOrder chunk_order(const Grid &g, bool d3, int chunk) {
  const int plane = g.nx * g.ny;
  if (!d3 || g.nz < 2 || plane % chunk != 0) return ChunkOrder{0, 0, 0};
  const int cpp = plane / chunk;
  int tile = 8;
  while (cpp % tile != 0) tile >>= 1;
  if (tile == cpp) return ChunkOrder{0, 0, 0};   // a tile would be the whole plane
  return ChunkOrder{cpp, tile, g.nz * tile};
}

// Unknowns per thread and chunk for storage type S: one 16-byte access.
template <typename S>
constexpr int vec_of() { return 16 / (int)sizeof(S); }

// ---------------------------------------------------------------------------
// Stencil
// ---------------------------------------------------------------------------

// Vector types for the non-temporal load/store builtins.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));

// V consecutive values held in FP64 registers; S is the storage type in memory
// (double, or float for the FP32-stored inner solver), converted on load/store.
// V is 1, 2 or 4; p is aligned to V elements.
template <int V, typename S = double>
struct Vals {
  double v[V];
  __device__ inline void load(const S *p) {
    if constexpr (sizeof(S) == 8 && V % 2 == 0) {
#pragma unroll
      for (int k = 0; k < V / 2; ++k) {
        const double2 t = reinterpret_cast<const double2 *>(p)[k];
        v[2 * k] = t.x;
        v[2 * k + 1] = t.y;
      }
    } else if constexpr (sizeof(S) == 4 && V == 4) {
      const float4 t = *reinterpret_cast<const float4 *>(p);
      v[0] = (double)t.x;
      v[1] = (double)t.y;
      v[2] = (double)t.z;
      v[3] = (double)t.w;
    } else if constexpr (sizeof(S) == 4 && V == 2) {
      const float2 t = *reinterpret_cast<const float2 *>(p);
      v[0] = (double)t.x;
      v[1] = (double)t.y;
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) v[k] = (double)p[k];
    }
  }
  __device__ inline void store(S *p) const {
    if constexpr (sizeof(S) == 8 && V % 2 == 0) {
#pragma unroll
      for (int k = 0; k < V / 2; ++k)
        reinterpret_cast<double2 *>(p)[k] = make_double2(v[2 * k], v[2 * k + 1]);
    } else if constexpr (sizeof(S) == 4 && V == 4) {
      *reinterpret_cast<float4 *>(p) =
          make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    } else if constexpr (sizeof(S) == 4 && V == 2) {
      *reinterpret_cast<float2 *>(p) = make_float2((float)v[0], (float)v[1]);
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) p[k] = (S)v[k];
    }
  }
  // The same accesses with the non-temporal hint.
  __device__ inline void load_nt(const S *p) {
    if constexpr (sizeof(S) == 8 && V % 2 == 0) {
#pragma unroll
      for (int k = 0; k < V / 2; ++k) {
        const nt_double2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_double2 *>(p) + k);
        v[2 * k] = t.x;
        v[2 * k + 1] = t.y;
      }
    } else if constexpr (sizeof(S) == 4 && V == 4) {
      const nt_float4 t = __builtin_nontemporal_load(reinterpret_cast<const nt_float4 *>(p));
      v[0] = (double)t.x;
      v[1] = (double)t.y;
      v[2] = (double)t.z;
      v[3] = (double)t.w;
    } else if constexpr (sizeof(S) == 4 && V == 2) {
      const nt_float2 t = __builtin_nontemporal_load(reinterpret_cast<const nt_float2 *>(p));
      v[0] = (double)t.x;
      v[1] = (double)t.y;
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) v[k] = (double)__builtin_nontemporal_load(p + k);
    }
  }
  __device__ inline void store_nt(S *p) const {
    if constexpr (sizeof(S) == 8 && V % 2 == 0) {
#pragma unroll
      for (int k = 0; k < V / 2; ++k)
        __builtin_nontemporal_store(nt_double2{v[2 * k], v[2 * k + 1]},
                                    reinterpret_cast<nt_double2 *>(p) + k);
    } else if constexpr (sizeof(S) == 4 && V == 4) {
      __builtin_nontemporal_store(nt_float4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]},
                                  reinterpret_cast<nt_float4 *>(p));
    } else if constexpr (sizeof(S) == 4 && V == 2) {
      __builtin_nontemporal_store(nt_float2{(float)v[0], (float)v[1]},
                                  reinterpret_cast<nt_float2 *>(p));
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) __builtin_nontemporal_store((S)v[k], p + k);
    }
  }
  template <bool NT>
  __device__ inline void ld(const S *p) {
    if constexpr (NT) load_nt(p); else load(p);
  }
  template <bool NT>
  __device__ inline void st(S *p) const {
    if constexpr (NT) store_nt(p); else store(p);
  }
  __device__ inline void zero() {
#pragma unroll
    for (int k = 0; k < V; ++k) v[k] = 0.0;
  }
};

// Sum of the face neighbours of unknown p (zero outside the grid), one load each.
template <bool D3, typename S = double>
__device__ inline double neighbour_sum(const S *z, int p, const Grid &g) {
  const int x = p % g.nx;
  const int rest = p / g.nx;
  const int y = D3 ? rest % g.ny : rest;
  double s = 0.0;
  if (x > 0) s += (double)z[p - 1];
  if (x < g.nx - 1) s += (double)z[p + 1];
  if (y > 0) s += (double)z[p - g.nx];
  if (y < g.ny - 1) s += (double)z[p + g.nx];
  if (D3) {
    const int zz = rest / g.ny;
    const int plane = g.nx * g.ny;
    if (zz > 0) s += (double)z[p - plane];
    if (zz < g.nz - 1) s += (double)z[p + plane];
  }
  return s;
}

// The values the stencil's FAST form reads beyond a thread's own V unknowns:
// the x-neighbours at the wave's edges (z[idx-1] for lane 0, z[idx+V] for lane
// 63) and the rows (and planes) above and below, with 16-byte loads.  Loaded
// apart from the arithmetic, so that a sweep can request them with its first
// chunk's own vectors, ahead of the scalar state.
template <int V, bool D3, typename S>
struct StencilHalo {
  double left, right;
  Vals<V, S> u, d;      // rows y-1, y+1
  Vals<V, S> f, b;      // planes z-1, z+1 (3D)
};

template <int V, bool D3, typename S>
__device__ inline void stencil_halo_load(const S *z, int idx, const Grid &g,
                                         StencilHalo<V, D3, S> &h) {
  const int x = idx % g.nx;
  const int rest = idx / g.nx;
  const int y = D3 ? rest % g.ny : rest;
  const int lane = threadIdx.x & 63;
  h.left = 0.0;
  h.right = 0.0;
  if (lane == 0 && x > 0) h.left = (double)z[idx - 1];
  if (lane == 63 && x + V < g.nx) h.right = (double)z[idx + V];
  if (y > 0) h.u.load(z + idx - g.nx);
  if (y < g.ny - 1) h.d.load(z + idx + g.nx);
  if constexpr (D3) {
    const int zz = rest / g.ny;
    const int plane = g.nx * g.ny;
    if (zz > 0) h.f.load(z + idx - plane);
    if (zz < g.nz - 1) h.b.load(z + idx + plane);
  }
}

// Where stencil_fast gets the values beyond a thread's own unknowns: loaded
// from the vector where they are used (the loop's chunks), or taken from a
// halo loaded ahead (a sweep's first chunk).  The same arithmetic either way.
template <int V, typename S>
struct RowsFromMemory {
  const S *z;
  __device__ inline double left(int idx) const { return (double)z[idx - 1]; }
  __device__ inline double right(int idx) const { return (double)z[idx + V]; }
  template <int W>   // 0: row above, 1: row below, 2: plane below, 3: plane above
  __device__ inline Vals<V, S> row(int q) const {
    Vals<V, S> r;
    r.load(z + q);
    return r;
  }
};

template <int V, bool D3, typename S>
struct RowsFromHalo {
  const StencilHalo<V, D3, S> &h;
  __device__ inline double left(int) const { return h.left; }
  __device__ inline double right(int) const { return h.right; }
  template <int W>
  __device__ inline const Vals<V, S> &row(int) const {
    if constexpr (W == 0) return h.u;
    else if constexpr (W == 1) return h.d;
    else if constexpr (W == 2) return h.f;
    else return h.b;
  }
};

// w = A z at a thread's V unknowns (a full chunk, nx a multiple of V: they
// share a row) from their values zc: x-neighbours from the thread's own values
// and the adjacent lanes (consecutive groups of V), the wave's edges, rows and
// planes from src.  Called by all 64 lanes together.
template <int V, bool D3, typename S, typename Src>
__device__ inline void stencil_fast(const Vals<V, S> &zc, int idx, const Grid &g, const Src &src,
                                    double (&w)[V]) {
  const double diag = D3 ? 6.0 : 4.0;
  const int x = idx % g.nx;
  const int rest = idx / g.nx;
  const int y = D3 ? rest % g.ny : rest;
  const int lane = threadIdx.x & 63;
  double left = lane_prev(zc.v[V - 1]);   // z[idx-1] held by the previous lane
  double right = lane_next(zc.v[0]);      // z[idx+V] held by the next lane
  if (lane == 0 && x > 0) left = src.left(idx);
  if (lane == 63 && x + V < g.nx) right = src.right(idx);
  double s[V];
#pragma unroll
  for (int k = 0; k < V; ++k)
    s[k] = (k > 0 ? zc.v[k - 1] : (x > 0 ? left : 0.0)) +
           (k < V - 1 ? zc.v[k + 1] : (x + V < g.nx ? right : 0.0));
  if (y > 0) {
    const Vals<V, S> u = src.template row<0>(idx - g.nx);
#pragma unroll
    for (int k = 0; k < V; ++k) s[k] += u.v[k];
  }
  if (y < g.ny - 1) {
    const Vals<V, S> d = src.template row<1>(idx + g.nx);
#pragma unroll
    for (int k = 0; k < V; ++k) s[k] += d.v[k];
  }
  if constexpr (D3) {
    const int zz = rest / g.ny;
    const int plane = g.nx * g.ny;
    if (zz > 0) {
      const Vals<V, S> f = src.template row<2>(idx - plane);
#pragma unroll
      for (int k = 0; k < V; ++k) s[k] += f.v[k];
    }
    if (zz < g.nz - 1) {
      const Vals<V, S> b = src.template row<3>(idx + plane);
#pragma unroll
      for (int k = 0; k < V; ++k) s[k] += b.v[k];
    }
  }
#pragma unroll
  for (int k = 0; k < V; ++k) w[k] = fma(diag, zc.v[k], -s[k]);
}

// w = A z at the V unknowns starting at idx, given their values zc.  FAST: a
// full chunk with nx a multiple of V; otherwise one unknown at a time, one load
// per neighbour.
template <int V, bool D3, bool FAST, typename S>
__device__ inline void apply_stencil(const S *z, int idx, const Vals<V, S> &zc, const Grid &g,
                                     double (&w)[V]) {
  if constexpr (FAST && V >= 2) {
    stencil_fast<V, D3, S>(zc, idx, g, RowsFromMemory<V, S>{z}, w);
  } else {
    const double diag = D3 ? 6.0 : 4.0;
#pragma unroll
    for (int v = 0; v < V; ++v) w[v] = fma(diag, zc.v[v], -neighbour_sum<D3, S>(z, idx + v, g));
  }
}

// ---------------------------------------------------------------------------
// Deterministic block reductions
// ---------------------------------------------------------------------------

// Sum over the 64 lanes of a wave, returned to every lane (called by all 64).
// Within each row of 16 lanes: neighbours (quad_perm [1,0,3,2]), pairs
// (quad_perm [2,3,0,1]), half-row mirror, row mirror - after each step every
// lane of the group holds the group's sum; then row 0's sum is added into row
// 1 and row 2's into row 3 (row_bcast:15), rows 0+1 into row 3 (row_bcast:31),
// and lane 63's total is broadcast.  Data-parallel-primitive moves instead of
// LDS permutes: a few cycles per step.  Fixed order, so the same bits each time.
__device__ inline double wave_sum(double v) {
  v += dpp_move<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);    // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);    // row_mirror
  v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 into rows 1, 3
  v += dpp_move<0x143, 0xC>(v);    // row_bcast:31 into rows 2, 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum acc[0..ND-1] over the workgroup; out[] (LDS) holds the result afterwards.
template <int ND>
__device__ inline void block_sum(const double (&acc)[ND], double *lds /* [4][ND] */,
                                 double *out /* [ND] */) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    const double s = wave_sum(acc[m]);
    if (lane == 0) lds[wave * ND + m] = s;
  }
  __syncthreads();
  if (threadIdx.x < ND) {
    const int m = threadIdx.x;
    out[m] = ((lds[m] + lds[ND + m]) + lds[2 * ND + m]) + lds[3 * ND + m];
  }
  __syncthreads();
}

// Grid-wide sums of the previous launch's partials, in a fixed order: thread j
// adds partials j, j + kThreads, ... of each product from zero, then the
// workgroup sums the threads' results.  The loads are split from the sums so a
// caller can request the partials together with its other loads (all of a
// thread's loads in flight at once: one memory round trip, not one per load).
// The loads are unconditional - every partial buffer holds ND rows of at least
// PER * kThreads entries, pstride apart - so the compiler can count them
// exactly and wait for an earlier load without waiting for these.  PER is
// kPartPer for kMaxStream workgroups, kSweepPer for the wider p(l)-CG sweeps.
constexpr int kPartPer = kMaxStream / kThreads;   // partials per product and thread
constexpr int kSweepPer = kSweepStream / kThreads;
static_assert(kMaxStream % kThreads == 0 && kSweepStream % kThreads == 0,
              "partials split evenly over the threads");

template <int ND, int PER = kPartPer>
struct PartRegs {
  double v[ND][PER];
};

template <int ND, int PER>
__device__ inline void partials_fetch(const double *part, int nparts, int pstride,
                                      PartRegs<ND, PER> &r) {
#pragma unroll
  for (int m = 0; m < ND; ++m)
#pragma unroll
    for (int j = 0; j < PER; ++j) r.v[m][j] = part[m * pstride + threadIdx.x + j * kThreads];
}

template <int ND, int PER>
__device__ inline void partials_sum(PartRegs<ND, PER> r, const double *part, int nparts,
                                    int pstride, double *lds, double *out) {
  // The values are taken as opaque here, so no addition is moved up to where
  // the loads were issued (the workgroup would wait for them there).
#pragma unroll
  for (int m = 0; m < ND; ++m)
#pragma unroll
    for (int j = 0; j < PER; ++j) asm volatile("" : "+v"(r.v[m][j]));
  double s[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if ((int)threadIdx.x + j * kThreads < nparts) acc += r.v[m][j];
    // More partials than PER * kThreads never occur; kept so any count sums right.
    for (int b = threadIdx.x + PER * kThreads; b < nparts; b += kThreads)
      acc += part[m * pstride + b];
    s[m] = acc;
  }
  block_sum<ND>(s, lds, out);
}

// The same sums where a kernel's streaming path sets its register budget: up to
// three products all loads in flight; beyond that one load at a time, since
// ND * kPartPer live values would raise the register count of the whole kernel
// (the batch tick's l >= 3 kernels: 76 -> 86 VGPRs at l = 3).  Same order.
template <int ND>
__device__ inline void sum_partials(const double *part, int nparts, int pstride, double *lds,
                                    double *out) {
  if constexpr (ND <= 3) {
    PartRegs<ND> r;
    partials_fetch<ND, kPartPer>(part, nparts, pstride, r);
    partials_sum<ND, kPartPer>(r, part, nparts, pstride, lds, out);
  } else {
    double s[ND];
#pragma unroll
    for (int m = 0; m < ND; ++m) {
      double acc = 0.0;
      for (int b = threadIdx.x; b < nparts; b += kThreads) acc += part[m * pstride + b];
      s[m] = acc;
    }
    block_sum<ND>(s, lds, out);
  }
}

// This workgroup's partials (index = streaming workgroup number).
template <int ND>
__device__ inline void store_partials(const double (&acc)[ND], double *part, int pstride,
                                      int slot, double *lds, double *blk) {
  block_sum<ND>(acc, lds, blk);
  if (threadIdx.x < ND) part[threadIdx.x * pstride + slot] = blk[threadIdx.x];
}

// Copy a scalar state (DevState, BatchState) between global memory and LDS (all
// threads).  Each thread requests its words before it writes any of them; the
// loads are unconditional (a thread past the end reads the last word again).
template <typename T>
struct WordRegs {
  static_assert(sizeof(T) % 8 == 0, "a state is copied in 8-byte words");
  static constexpr int kWords = (int)(sizeof(T) / 8);
  static constexpr int kPer = (kWords + kThreads - 1) / kThreads;
  double v[kPer];
};

template <typename T>
__device__ inline void words_fetch(const T *src, WordRegs<T> &r) {
  const double *s = reinterpret_cast<const double *>(src);
#pragma unroll
  for (int j = 0; j < WordRegs<T>::kPer; ++j) {
    const int k = threadIdx.x + j * kThreads;
    r.v[j] = s[k < WordRegs<T>::kWords ? k : WordRegs<T>::kWords - 1];
  }
}

template <typename T>
__device__ inline void words_put(const WordRegs<T> &r, T *dst) {
  double *d = reinterpret_cast<double *>(dst);
#pragma unroll
  for (int j = 0; j < WordRegs<T>::kPer; ++j) {
    const int k = threadIdx.x + j * kThreads;
    if (k < WordRegs<T>::kWords) d[k] = r.v[j];
  }
  __syncthreads();
}

__device__ inline void state_load(const DevState *st, DevState *sh) {
  WordRegs<DevState> r;
  words_fetch(st, r);
  words_put(r, sh);
}
__device__ inline void state_store(const DevState *sh, DevState *st) {
  __syncthreads();
  const double *src = reinterpret_cast<const double *>(sh);
  double *dst = reinterpret_cast<double *>(st);
  for (int k = threadIdx.x; k < (int)(sizeof(DevState) / 8); k += kThreads) dst[k] = src[k];
}

// Progress for the host (visible there at the latest when the kernel ends).
__device__ inline void publish(const DevState &s, HostStatus *hs, double zeta, int seq) {
  hs->status = s.status;
  hs->last_t = s.last_t;
  hs->cols = s.cols;
  hs->seq = seq;
  hs->zeta = zeta;
  hs->beta = s.beta;
  hs->rref = s.rref;
  hs->sumsq = s.sumsq;
}

// ---------------------------------------------------------------------------
// Scalar engine of p(l)-CG: one column of G, one column of T, one LU step
// ---------------------------------------------------------------------------

__host__ __device__ inline double &gref(DevState &s, int r, int c) {
  return s.g[c % kGRing][r - c + 2 * kLMax];
}

// Column c of G from the raw products raw[0] = (z_c, v_{c-l}) and
// raw[m] = (z_c, z_{c-l+m}), m = 1..l: the entries below the l-th upper
// diagonal from Eq. (symmetry_G), the forward substitution for rows
// c-l+1 .. c-1 and the square root for the diagonal (Alg. 1, update of G);
// then gamma_t, delta_t (Eqs. haa1, haa3) and eta_t, zeta_t (Eq. LU and the
// recursion for zeta) for t = c-1, and the breakdown / convergence tests.
// Runs in one thread.  This is the form for any l; the kernels run
// engine_column_l<L> below, which a host replay test checks against it, state
// byte for state byte, on recorded dot-product streams.
__host__ __device__ inline void engine_column(DevState &s, const double *raw, int c,
                                              double *hist) {
  const int l = s.l;
  const int t = c - 1;
  const int lo = c - 2 * l > 0 ? c - 2 * l : 0;
  for (int r = c - 2 * l; r <= c; ++r) gref(s, r, c) = 0.0;
  for (int r = lo; r <= c - l - 1; ++r) gref(s, r, c) = gref(s, c - l, r + l);
  if (c - l >= 0) gref(s, c - l, c) = raw[0];
  for (int m = 1; m <= l; ++m) {
    const int j = c - l + m;
    if (j >= 0) gref(s, j, c) = raw[m];
  }
  const int jlo = c - l + 1 > 0 ? c - l + 1 : 0;
  for (int j = jlo; j < c; ++j) {
    double v = gref(s, j, c);
    for (int k = lo; k < j; ++k) v -= gref(s, k, j) * gref(s, k, c);
    gref(s, j, c) = v / gref(s, j, j);
  }
  double arg = gref(s, c, c);
  for (int k = lo; k < c; ++k) arg -= gref(s, k, c) * gref(s, k, c);
  bool broken = !(isfinite(arg) && arg > 0.0);
  double gam = 0.0, dlt = 0.0, eta = 0.0, zeta = 0.0;
  if (!broken) {
    gref(s, c, c) = sqrt(arg);
    const double gtt = gref(s, t, t);
    const double corr = t >= 1 ? gref(s, t - 1, t) * s.dlt[(t - 1) % kTRing] : 0.0;
    if (t < l) {
      gam = (gref(s, t, c) + s.sigma[t] * gtt - corr) / gtt;
      dlt = gref(s, c, c) / gtt;
    } else {
      gam = (gtt * s.gam[(t - l) % kTRing] + gref(s, t, c) * s.dlt[(t - l) % kTRing] - corr) / gtt;
      dlt = (gref(s, c, c) * s.dlt[(t - l) % kTRing]) / gtt;
    }
    broken = !(isfinite(gam) && isfinite(dlt) && dlt > 0.0);
    if (!broken) {
      if (t == 0) {
        eta = gam;
        zeta = s.beta;
      } else {
        const double lam = s.dlt[(t - 1) % kTRing] / s.eta[(t - 1) % kTRing];
        eta = gam - lam * s.dlt[(t - 1) % kTRing];
        zeta = -lam * s.zeta[(t - 1) % kTRing];
      }
      broken = !(isfinite(eta) && eta > 0.0 && isfinite(zeta));
    }
  }
  s.cols = c;
  if (broken) {
    s.status = kBroken;
    s.last_t = t - 1;
    return;
  }
  s.gam[t % kTRing] = gam;
  s.dlt[t % kTRing] = dlt;
  s.eta[t % kTRing] = eta;
  s.zeta[t % kTRing] = zeta;
  if (hist != nullptr && t < s.hist_cap) {
    hist[4 * t + 0] = gam;
    hist[4 * t + 1] = dlt;
    hist[4 * t + 2] = eta;
    hist[4 * t + 3] = zeta;
  }
  if (t >= 1 && fabs(zeta) < s.abs_tol) {
    s.status = kConverged;
    s.last_t = t;
  }
}

// engine_column for a pipeline length L known at compile time: the same
// operations on the same operands in the same order (so the same bits), with
// the new column c held in registers (row r at gc[r - c + 2L]) instead of
// being written and re-read through the state's G ring, and stored once at the
// end.  Finalised columns are only read, so their loads need not wait for the
// new column's updates.
// The column step for l = 1, the step every p(1)-CG workgroup runs before it
// streams, in two parts: engine_gather_1 reads every entry of the state the
// column may use (indices clamped into range; what a branch does not take goes
// unused), engine_column_1 computes with the same expressions as the general
// form below.  A kernel can so issue all reads of its LDS copy together (and
// make sure of it between the two calls) instead of one per branch.
struct EngineIn1 {
  double g_tt;     // g_{c-1,c-1}: the symmetric entry g_{c-1,c-1} of column c and g_{t,t}
  double g_pt;     // g_{t-1,t}
  double dlt1, gam1, eta1, zeta1;   // entries t-1 of the rings
  double sigma0, beta, abs_tol;
  int hist_cap;
};

__host__ __device__ inline EngineIn1 engine_gather_1(const DevState &s, int c) {
  const int t = c - 1;
  const int tp = t >= 1 ? t - 1 : 0;
  EngineIn1 in;
  in.g_tt = s.g[((c - 1) % kGRing + kGRing) % kGRing][2 * kLMax];
  in.g_pt = s.g[(t % kGRing + kGRing) % kGRing][tp - t + 2 * kLMax];
  in.dlt1 = s.dlt[tp % kTRing];
  in.gam1 = s.gam[tp % kTRing];
  in.eta1 = s.eta[tp % kTRing];
  in.zeta1 = s.zeta[tp % kTRing];
  in.sigma0 = s.sigma[0];
  in.beta = s.beta;
  in.abs_tol = s.abs_tol;
  in.hist_cap = s.hist_cap;
  return in;
}

__host__ __device__ inline void engine_column_1(DevState &s, const EngineIn1 &in,
                                                const double *raw, int c, double *hist) {
  const int t = c - 1;
  double gc[3];
  gc[0] = c - 2 >= 0 ? in.g_tt : 0.0;
  gc[1] = c - 1 >= 0 ? raw[0] : 0.0;
  gc[2] = c >= 0 ? raw[1] : 0.0;
  double arg = gc[2];
  if (c - 2 >= 0) arg -= gc[0] * gc[0];
  if (c - 1 >= 0) arg -= gc[1] * gc[1];
  bool broken = !(isfinite(arg) && arg > 0.0);
  double gam = 0.0, dlt = 0.0, eta = 0.0, zeta = 0.0;
  if (!broken) {
    gc[2] = sqrt(arg);
    const double gtt = in.g_tt;
    const double corr = t >= 1 ? in.g_pt * in.dlt1 : 0.0;
    if (t < 1) {
      gam = (gc[1] + in.sigma0 * gtt - corr) / gtt;
      dlt = gc[2] / gtt;
    } else {
      gam = (gtt * in.gam1 + gc[1] * in.dlt1 - corr) / gtt;
      dlt = (gc[2] * in.dlt1) / gtt;
    }
    broken = !(isfinite(gam) && isfinite(dlt) && dlt > 0.0);
    if (!broken) {
      if (t == 0) {
        eta = gam;
        zeta = in.beta;
      } else {
        const double lam = in.dlt1 / in.eta1;
        eta = gam - lam * in.dlt1;
        zeta = -lam * in.zeta1;
      }
      broken = !(isfinite(eta) && eta > 0.0 && isfinite(zeta));
    }
  }
  for (int q = 0; q < 3; ++q) gref(s, c - 2 + q, c) = gc[q];
  s.cols = c;
  if (broken) {
    s.status = kBroken;
    s.last_t = t - 1;
    return;
  }
  s.gam[t % kTRing] = gam;
  s.dlt[t % kTRing] = dlt;
  s.eta[t % kTRing] = eta;
  s.zeta[t % kTRing] = zeta;
  if (hist != nullptr && t < in.hist_cap) {
    hist[4 * t + 0] = gam;
    hist[4 * t + 1] = dlt;
    hist[4 * t + 2] = eta;
    hist[4 * t + 3] = zeta;
  }
  if (t >= 1 && fabs(zeta) < in.abs_tol) {
    s.status = kConverged;
    s.last_t = t;
  }
}

template <int L>
__host__ __device__ inline void engine_column_l(DevState &s, const double *raw, int c,
                                                double *hist) {
  constexpr int W = 2 * L + 1;
  const int t = c - 1;
  if constexpr (L == 1) {
    engine_column_1(s, engine_gather_1(s, c), raw, c, hist);
    return;
  }
  double gc[W];
#pragma unroll
  for (int q = 0; q < W; ++q) gc[q] = 0.0;
  // rows r = c-2L .. c-L-1 from Eq. (symmetry_G): g_{r,c} = g_{c-L, r+L}
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int r = c - 2 * L + q;
    if (r >= 0) gc[q] = gref(s, c - L, r + L);
  }
  if (c - L >= 0) gc[L] = raw[0];
#pragma unroll
  for (int m = 1; m <= L; ++m)
    if (c - L + m >= 0) gc[L + m] = raw[m];
  // forward substitution for rows j = c-L+1 .. c-1, in increasing j
#pragma unroll
  for (int m = 1; m < L; ++m) {
    const int j = c - L + m;
    if (j < 0) continue;
    double v = gc[L + m];
#pragma unroll
    for (int q = 0; q < L + m; ++q) {
      const int k = c - 2 * L + q;
      if (k >= 0) v -= gref(s, k, j) * gc[q];
    }
    gc[L + m] = v / gref(s, j, j);
  }
  double arg = gc[2 * L];
#pragma unroll
  for (int q = 0; q < 2 * L; ++q) {
    const int k = c - 2 * L + q;
    if (k >= 0) arg -= gc[q] * gc[q];
  }
  bool broken = !(isfinite(arg) && arg > 0.0);
  double gam = 0.0, dlt = 0.0, eta = 0.0, zeta = 0.0;
  if (!broken) {
    gc[2 * L] = sqrt(arg);
    const double gtt = gref(s, t, t);
    const double corr = t >= 1 ? gref(s, t - 1, t) * s.dlt[(t - 1) % kTRing] : 0.0;
    if (t < L) {
      gam = (gc[2 * L - 1] + s.sigma[t] * gtt - corr) / gtt;
      dlt = gc[2 * L] / gtt;
    } else {
      gam = (gtt * s.gam[(t - L) % kTRing] + gc[2 * L - 1] * s.dlt[(t - L) % kTRing] - corr) / gtt;
      dlt = (gc[2 * L] * s.dlt[(t - L) % kTRing]) / gtt;
    }
    broken = !(isfinite(gam) && isfinite(dlt) && dlt > 0.0);
    if (!broken) {
      if (t == 0) {
        eta = gam;
        zeta = s.beta;
      } else {
        const double lam = s.dlt[(t - 1) % kTRing] / s.eta[(t - 1) % kTRing];
        eta = gam - lam * s.dlt[(t - 1) % kTRing];
        zeta = -lam * s.zeta[(t - 1) % kTRing];
      }
      broken = !(isfinite(eta) && eta > 0.0 && isfinite(zeta));
    }
  }
#pragma unroll
  for (int q = 0; q < W; ++q) gref(s, c - 2 * L + q, c) = gc[q];
  s.cols = c;
  if (broken) {
    s.status = kBroken;
    s.last_t = t - 1;
    return;
  }
  s.gam[t % kTRing] = gam;
  s.dlt[t % kTRing] = dlt;
  s.eta[t % kTRing] = eta;
  s.zeta[t % kTRing] = zeta;
  if (hist != nullptr && t < s.hist_cap) {
    hist[4 * t + 0] = gam;
    hist[4 * t + 1] = dlt;
    hist[4 * t + 2] = eta;
    hist[4 * t + 3] = zeta;
  }
  if (t >= 1 && fabs(zeta) < s.abs_tol) {
    s.status = kConverged;
    s.last_t = t;
  }
}

// ---------------------------------------------------------------------------
// Coefficients of one sweep
// ---------------------------------------------------------------------------

template <int L>
struct Coef {
  double gam, dm1, inv_del, inv_eta, zm1, zm2, sigma_i;
  double sig[L];
};

// Every entry is read whatever t is (ring indices clamped into range, entries a
// sweep does not use replaced by zero afterwards), so that a workgroup reading
// s from global memory issues all its loads at once: one round trip, where
// loads under conditions on t took up to three dependent ones.
template <int L>
__device__ inline void read_coef(const DevState &s, int i, int t, Coef<L> &cf) {
  const int t0 = (t >= 0 ? t : 0) % kTRing;
  const int t1 = (t >= 1 ? t - 1 : 0) % kTRing;
  const int t2 = (t >= 2 ? t - 2 : 0) % kTRing;
  const double gam = s.gam[t0], dlt = s.dlt[t0], dlt1 = s.dlt[t1], eta = s.eta[t0];
  const double zeta1 = s.zeta[t1], zeta2 = s.zeta[t2];
  const double sigma_i = s.sigma[i >= 0 && i < kLMax ? i : 0];
  double sig[L];
#pragma unroll
  for (int k = 0; k < L; ++k) sig[k] = s.sigma[k];
  cf.gam = t >= 0 ? gam : 0.0;
  cf.inv_del = t >= 0 ? 1.0 / dlt : 0.0;
  cf.dm1 = t >= 1 ? dlt1 : 0.0;
  cf.inv_eta = t >= 0 ? 1.0 / eta : 0.0;
  cf.zm1 = t >= 1 ? zeta1 : 0.0;
  cf.zm2 = t >= 2 ? zeta2 : 0.0;
  cf.sigma_i = t >= 0 ? 0.0 : sigma_i;
#pragma unroll
  for (int k = 0; k < L; ++k) cf.sig[k] = sig[k];
}

// The unscaled integer Dirichlet Laplacian (5-point in 2D, 7-point in 3D).
// Every operator also offers its FAST form split in two: halo_load requests
// what the operator reads beyond a thread's own unknowns (Halo<V>), apply_halo
// forms w from it, with the arithmetic of apply<V, true>.  A sweep uses the
// split to request its first chunk's operator data ahead of the scalar state.
// Operators whose FAST form is not split have an empty halo, and apply_halo
// is apply<V, true>.
struct NoHalo {};

// The 3D stencil's halo is not split: its four rows and planes held ahead
// took the p(3) sweep to 135 registers (three waves per SIMD).
template <bool D3, typename S>
struct ConstOp {
  Grid g;
  template <int V>
  using Halo = std::conditional_t<D3, NoHalo, StencilHalo<V, false, S>>;
  template <int V, bool FAST>
  __device__ inline void apply(const S *z, int idx, const Vals<V, S> &zc, double (&w)[V]) const {
    apply_stencil<V, D3, FAST, S>(z, idx, zc, g, w);
  }
  template <int V>
  __device__ inline void halo_load(const S *z, int idx, Halo<V> &h) const {
    if constexpr (!D3) stencil_halo_load<V, false, S>(z, idx, g, h);
  }
  template <int V>
  __device__ inline void apply_halo(const S *z, int idx, const Vals<V, S> &zc, const Halo<V> &h,
                                    double (&w)[V]) const {
    if constexpr (D3)
      apply_stencil<V, true, true, S>(z, idx, zc, g, w);
    else
      stencil_fast<V, false, S>(zc, idx, g, RowsFromHalo<V, false, S>{h}, w);
  }
};

// Diagonal operator, (A z)_p = d_p z_p with d in FP64: the one-point stencil of
// the paper's communication-bound toy problem (Sec. 4.2), a diagonal matrix
// holding the spectrum of the 2D Laplacian.  One extra FP64 read per unknown.
template <typename S>
struct DiagOp {
  const double *d;
  template <int V>
  using Halo = Vals<V, double>;   // the diagonal entries
  template <int V, bool FAST>
  __device__ inline void apply(const S *, int idx, const Vals<V, S> &zc, double (&w)[V]) const {
    Vals<V, double> dv;
    dv.load(d + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) w[v] = dv.v[v] * zc.v[v];
  }
  template <int V>
  __device__ inline void halo_load(const S *, int idx, Halo<V> &h) const {
    h.load(d + idx);
  }
  template <int V>
  __device__ inline void apply_halo(const S *, int, const Vals<V, S> &zc, const Halo<V> &h,
                                    double (&w)[V]) const {
#pragma unroll
    for (int v = 0; v < V; ++v) w[v] = h.v[v] * zc.v[v];
  }
};

// General sparse operator in CSR form, one row per unknown: (A z)_p = sum over
// the stored entries j of row p of va[j] * z[ci[j]] (FP64 values, stored
// order).  With ell_k > 0 the entries come from the padded column-major ELL
// copy instead (entry j of row p at j * ell_ld + p): consecutive rows are then
// read by consecutive lanes, one coalesced access per entry index for the V
// rows of a thread.  Both forms add the same products in the same order
// (padding adds exact zeros).
template <typename S, bool NT = false>
struct CsrOp {
  const int64_t *rp;
  const int32_t *ci;
  const double *va;
  int ell_k, ell_ld;
  template <int V>
  using Halo = NoHalo;
  template <int V>
  __device__ inline void halo_load(const S *, int, Halo<V> &) const {}
  template <int V>
  __device__ inline void apply_halo(const S *z, int idx, const Vals<V, S> &zc, const Halo<V> &,
                                    double (&w)[V]) const {
    apply<V, true>(z, idx, zc, w);
  }
  __device__ inline double row(const S *z, int p) const {
    double s = 0.0;
    if (ell_k > 0) {
      for (int j = 0; j < ell_k; ++j) {
        const size_t e = (size_t)j * ell_ld + p;
        s = fma(va[e], (double)z[ci[e]], s);
      }
    } else {
      const int64_t e = rp[p + 1];
      for (int64_t j = rp[p]; j < e; ++j) s = fma(va[j], (double)z[ci[j]], s);
    }
    return s;
  }
  template <int V, bool FAST>
  __device__ inline void apply(const S *z, int idx, const Vals<V, S> &, double (&w)[V]) const {
    if (ell_k > 0 && V >= 2) {
      // idx is a multiple of V and ell_ld of 4: aligned vector accesses
#pragma unroll
      for (int v = 0; v < V; ++v) w[v] = 0.0;
      for (int j = 0; j < ell_k; ++j) {
        const size_t e = (size_t)j * ell_ld + idx;
        Vals<V, double> vv;
        vv.template ld<NT>(va + e);
        int c[V];
        if constexpr (V == 2) {
          const int2 t = *reinterpret_cast<const int2 *>(ci + e);
          c[0] = t.x;
          c[1] = t.y;
        } else if constexpr (V == 4) {
          const int4 t = *reinterpret_cast<const int4 *>(ci + e);
          c[0] = t.x;
          c[1] = t.y;
          c[2] = t.z;
          c[3] = t.w;
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) c[v] = ci[e + v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) w[v] = fma(vv.v[v], (double)z[c[v]], w[v]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) w[v] = row(z, idx + v);
    }
  }
};

// Variable-coefficient grid operator at unknown p: d_p u_p - sum over the
// interior edges (p, q) of w_pq u_q (u stored as T, weights and arithmetic
// FP64).  Jacobi-scaled form (dg NULL): unit diagonal and w_pq = c_pq /
// sqrt(d_p d_q); unscaled form: dg = d (the sum of the edges at p, boundary
// edges included) and w_pq = c_pq.  Edge layout: sx per row (y, z) nx+1 values
// (edge left of x at index x), sy per plane ny+1 rows of nx (edge below y at
// row y), sz nz+1 planes (edge below z at plane z).
struct VarOp {
  const double *sx, *sy, *sz;
  int n, nx, ny, nz, d3;
  const double *dg;
  template <int V>
  using Halo = NoHalo;
  template <int V, typename S>
  __device__ inline void halo_load(const S *, int, Halo<V> &) const {}
  template <int V, typename S>
  __device__ inline void apply_halo(const S *z, int idx, const Vals<V, S> &zc, const Halo<V> &,
                                    double (&w)[V]) const {
    apply<V, true, S>(z, idx, zc, w);
  }
  // The operator at p with the value at p given and the others read through
  // get(q) (a vector, or values formed on the fly).
  template <typename F>
  __device__ inline double at_f(int p, double up, F get) const {
    const int x = p % nx;
    const int rest = p / nx;
    const int y = d3 ? rest % ny : rest;
    double s = 0.0;
    const int xe = rest * (nx + 1) + x;          // edge left of p in its row
    if (x > 0) s = fma(sx[xe], get(p - 1), s);
    if (x < nx - 1) s = fma(sx[xe + 1], get(p + 1), s);
    const int z = d3 ? rest / ny : 0;
    const int ye = p + z * nx;                   // edge below p in its column
    if (y > 0) s = fma(sy[ye], get(p - nx), s);
    if (y < ny - 1) s = fma(sy[ye + nx], get(p + nx), s);
    if (d3) {
      const int plane = nx * ny;
      if (z > 0) s = fma(sz[p], get(p - plane), s);
      if (z < nz - 1) s = fma(sz[p + plane], get(p + plane), s);
    }
    return dg != nullptr ? fma(dg[p], up, -s) : up - s;
  }
  template <typename T>
  __device__ inline double at(const T *u, int p) const {
    return at_f(p, (double)u[p], [u](int q) { return (double)u[q]; });
  }
  // FAST (a full chunk, nx a multiple of V): the thread's V unknowns share a
  // row; x-neighbours come from its own values and the adjacent lanes, the rows
  // and planes above and below and the y/z edge weights with 16-byte accesses.
  // Each unknown's terms are added in the order of at().
  template <int V, bool FAST, typename S>
  __device__ inline void apply(const S *z, int idx, const Vals<V, S> &zc,
                               double (&w)[V]) const {
    if constexpr (FAST && V >= 2) {
      const int x = idx % nx;
      const int rest = idx / nx;
      const int y = d3 ? rest % ny : rest;
      const int zz = d3 ? rest / ny : 0;
      const int plane = nx * ny;
      const int lane = threadIdx.x & 63;
      double left = lane_prev(zc.v[V - 1]);    // z[idx-1] held by the previous lane
      double right = lane_next(zc.v[0]);       // z[idx+V] held by the next lane
      if (lane == 0 && x > 0) left = (double)z[idx - 1];
      if (lane == 63 && x + V < nx) right = (double)z[idx + V];
      const int xe = rest * (nx + 1) + x;             // edge left of idx in its row
      const int ye = idx + zz * nx;                   // edge below idx in its column
      // one neighbour direction at a time (few values live at once); each
      // unknown's sum still takes its terms in the order of at()
      double s[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        s[k] = 0.0;
        if (x + k > 0) s[k] = fma(sx[xe + k], k > 0 ? zc.v[k - 1] : left, s[k]);
        if (x + k < nx - 1) s[k] = fma(sx[xe + k + 1], k < V - 1 ? zc.v[k + 1] : right, s[k]);
      }
      if (y > 0) {
        Vals<V, S> u;
        Vals<V, double> c;
        u.load(z + idx - nx);
        c.load(sy + ye);
#pragma unroll
        for (int k = 0; k < V; ++k) s[k] += c.v[k] * u.v[k];
      }
      if (y < ny - 1) {
        Vals<V, S> u;
        Vals<V, double> c;
        u.load(z + idx + nx);
        c.load(sy + ye + nx);
#pragma unroll
        for (int k = 0; k < V; ++k) s[k] += c.v[k] * u.v[k];
      }
      if (d3 && zz > 0) {
        Vals<V, S> u;
        Vals<V, double> c;
        u.load(z + idx - plane);
        c.load(sz + idx);
#pragma unroll
        for (int k = 0; k < V; ++k) s[k] += c.v[k] * u.v[k];
      }
      if (d3 && zz < nz - 1) {
        Vals<V, S> u;
        Vals<V, double> c;
        u.load(z + idx + plane);
        c.load(sz + idx + plane);
#pragma unroll
        for (int k = 0; k < V; ++k) s[k] += c.v[k] * u.v[k];
      }
      if (dg != nullptr) {
        Vals<V, double> dv;
        dv.load(dg + idx);
#pragma unroll
        for (int k = 0; k < V; ++k) w[k] = fma(dv.v[k], zc.v[k], -s[k]);
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k) w[k] = zc.v[k] - s[k];
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) w[v] = at(z, idx + v);
    }
  }
};

// ---------------------------------------------------------------------------
// p(l)-CG sweep: iteration i of Alg. 1
// ---------------------------------------------------------------------------

// The recurrences of one p(l)-CG iteration for V consecutive unknowns.  Op is
// the operator: Op::apply<V, FAST>(z, idx, zc, w) sets w = A z at idx .. idx+V-1.
// PAIR: p in two buffers, x written on even t only (a.xmode kXSkip / kXPair);
// else p in place and x written in every sweep.
template <int L, typename S, typename Op, int H = 0, bool PAIR = false>
struct Sweep {
  using Args = SweepArgsT<S>;
  static constexpr int ND = L + 1;
  static constexpr bool NTL = (H & kHintLoads) != 0;
  static constexpr bool NTS = (H & kHintStores) != 0;

  // The vectors a steady-state step reads at its own unknowns (the operator
  // reads its neighbours itself), loaded ahead of the step: the sweeps of
  // l <= 3 request their first chunk's before they read the scalar state (no
  // older z^{(l)} vectors are read for these l).
  template <int V>
  struct Loads {
    Vals<V, S> zc, zp, ck[L], pk[L], pv, xv, qv;
    typename Op::template Halo<V> halo;   // the operator's data beyond the own unknowns
  };
  template <int V>
  __device__ static inline void steady_load(const Args &a, const Op &op, int idx, int t,
                                            Loads<V> &d) {
    static_assert(L <= 3, "older z^(l) vectors are not preloaded");
    d.zc.load(a.zl[0] + idx);
    op.template halo_load<V>(a.zl[0], idx, d.halo);
    d.zp.template ld<NTL>(a.zl[1] + idx);
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
      d.ck[k].template ld<NTL>(a.zk_cur[k] + idx);
      if (t >= 1) d.pk[k].template ld<NTL>(a.zk_prev[k] + idx); else d.pk[k].zero();
    }
    if (t >= 1) {
      d.pv.template ld<NTL>(a.p + idx);
      if constexpr (!PAIR) {
        d.xv.template ld<NTL>(a.x + idx);
      } else if (a.xmode != kXSkip) {
        d.xv.template ld<NTL>(a.x + idx);
        if (a.xmode == kXPair) d.qv.template ld<NTL>(a.p_out + idx);
      }
    }
  }

  // Steady state, i >= l: K1 (SpMV of z^{(l)}_i), K4 (all basis recurrences,
  // Eqs. all_z_rec2 and specific_z_rec), K6 (p_t, x_t; Eqs. pdir, x_a2) and
  // K5 (the l+1 products that start column i+1 of G).  PRE: the vectors read at
  // the step's own unknowns come from *pre (steady_load) instead of memory;
  // the arithmetic is the same.
  template <int V, bool FAST, bool PRE = false>
  __device__ static inline void steady(const Args &a, const Op &op, int idx, int t,
                                       const Coef<L> &cf, double (&acc)[ND],
                                       const Loads<V> *pre = nullptr) {
    Vals<V, S> zc, zp;
    if constexpr (PRE) {
      zc = pre->zc;
      zp = pre->zp;
    } else {
      zc.load(a.zl[0] + idx);
      zp.template ld<NTL>(a.zl[1] + idx);
    }
    double w[V];
    if constexpr (PRE)
      op.template apply_halo<V>(a.zl[0], idx, zc, pre->halo, w);
    else
      op.template apply<V, FAST>(a.zl[0], idx, zc, w);
    double zn[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
      zn[v] = fma(-cf.dm1, zp.v[v], fma(-cf.gam, zc.v[v], w[v])) * cf.inv_del;
    // Products with older z^{(l)} vectors, read before zl_out (the slot of
    // z^{(l)}_{i+1-R}) is overwritten below.
#pragma unroll
    for (int m = 1; m <= L - 3; ++m) {
      Vals<V, S> zh;
      zh.template ld<NTL>(a.zl[L - 1 - m] + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[m] = fma(zn[v], zh.v[v], acc[m]);
    }
    double above[V], vt[V], vnew[V];
#pragma unroll
    for (int v = 0; v < V; ++v) above[v] = zc.v[v];
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
      Vals<V, S> ck, pk;
      if constexpr (PRE) {
        ck = pre->ck[k];
        pk = pre->pk[k];
      } else {
        ck.template ld<NTL>(a.zk_cur[k] + idx);
        if (t >= 1) pk.template ld<NTL>(a.zk_prev[k] + idx); else pk.zero();
      }
      Vals<V, S> nk;
      const double sk = cf.sig[k] - cf.gam;
#pragma unroll
      for (int v = 0; v < V; ++v)
        nk.v[v] = fma(-cf.dm1, pk.v[v], fma(sk, ck.v[v], above[v])) * cf.inv_del;
      nk.template st<NTS>(a.zk_prev[k] + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) above[v] = ck.v[v];
      if (k == 0) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          vt[v] = ck.v[v];
          vnew[v] = nk.v[v];
        }
      }
    }
    Vals<V, S> pv;
    if (t == 0) {
#pragma unroll
      for (int v = 0; v < V; ++v) pv.v[v] = vt[v] * cf.inv_eta;
    } else if constexpr (!PAIR) {
      Vals<V, S> xv;
      if constexpr (PRE) {
        pv = pre->pv;
        xv = pre->xv;
      } else {
        pv.template ld<NTL>(a.p + idx);
        xv.template ld<NTL>(a.x + idx);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xv.v[v] = fma(cf.zm1, pv.v[v], xv.v[v]);
        pv.v[v] = fma(-cf.dm1, pv.v[v], vt[v]) * cf.inv_eta;
      }
      xv.template st<NTS>(a.x + idx);
    } else {
      if constexpr (PRE) pv = pre->pv; else pv.template ld<NTL>(a.p + idx);
      if (a.xmode != kXSkip) {
        Vals<V, S> xv;
        if constexpr (PRE) xv = pre->xv; else xv.template ld<NTL>(a.x + idx);
        if (a.xmode == kXPair) {
          // x_{t-1} = x_{t-2} + zeta_{t-2} p_{t-2}, rounded to S as if stored;
          // p_{t-2} sits in the buffer that receives p_t below
          Vals<V, S> qv;
          if constexpr (PRE) qv = pre->qv; else qv.template ld<NTL>(a.p_out + idx);
#pragma unroll
          for (int v = 0; v < V; ++v) xv.v[v] = (double)(S)fma(cf.zm2, qv.v[v], xv.v[v]);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) xv.v[v] = fma(cf.zm1, pv.v[v], xv.v[v]);
        xv.template st<NTS>(a.x + idx);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) pv.v[v] = fma(-cf.dm1, pv.v[v], vt[v]) * cf.inv_eta;
    }
    pv.template st<NTS>((PAIR ? a.p_out : a.p) + idx);
    Vals<V, S> out;
#pragma unroll
    for (int v = 0; v < V; ++v) out.v[v] = zn[v];
    out.template st<NTS>(a.zl_out + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[0] = fma(zn[v], vnew[v], acc[0]);                     // (z_{i+1}, v_{t+1})
      acc[L] = fma(zn[v], zn[v], acc[L]);                       // (z_{i+1}, z_{i+1})
      if (L >= 2) acc[L - 1] = fma(zn[v], zc.v[v], acc[L - 1]); // (z_{i+1}, z_i)
      if (L >= 3) acc[L - 2] = fma(zn[v], zp.v[v], acc[L - 2]); // (z_{i+1}, z_{i-1})
    }
  }

  // Start-up, i < l: z^{(l)}_{i+1} = (A - sigma_i) z^{(l)}_i, copied into basis
  // i+1; products (z_{i+1}, z_j), j >= 0, and (z_l, v_0) when i = l-1.
  template <int V, bool FAST>
  __device__ static inline void startup(const Args &a, const Op &op, int idx, int i,
                                        double sigma_i, double (&acc)[ND]) {
    Vals<V, S> zc;
    zc.load(a.zl[0] + idx);
    double w[V];
    op.template apply<V, FAST>(a.zl[0], idx, zc, w);
    Vals<V, S> zn;
#pragma unroll
    for (int v = 0; v < V; ++v) zn.v[v] = fma(-sigma_i, zc.v[v], w[v]);
#pragma unroll
    for (int m = 1; m <= L - 2; ++m) {
      const int h = L - 1 - m;
      if (h <= i) {
        Vals<V, S> zh;
        zh.template ld<NTL>(a.zl[h] + idx);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[m] = fma(zn.v[v], zh.v[v], acc[m]);
      }
    }
    if (a.v0 != nullptr) {
      Vals<V, S> vz;
      vz.template ld<NTL>(a.v0 + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[0] = fma(zn.v[v], vz.v[v], acc[0]);
    }
    zn.template st<NTS>(a.zl_out + idx);
    if (a.copy_dst != nullptr) zn.template st<NTS>(a.copy_dst + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[L] = fma(zn.v[v], zn.v[v], acc[L]);
      if (L >= 2) acc[L - 1] = fma(zn.v[v], zc.v[v], acc[L - 1]);
    }
  }

  // The V unknowns idx .. idx+V-1 of a thread (one at a time past the end of
  // a ragged last chunk).
  template <int V, bool FAST>
  __device__ static inline void chunk(const Args &a, const Op &op, int idx, int t,
                                      const Coef<L> &cf, double (&acc)[ND]) {
    if (idx + V <= a.n) {
      if (t >= 0)
        steady<V, FAST>(a, op, idx, t, cf, acc);
      else
        startup<V, FAST>(a, op, idx, a.i, cf.sigma_i, acc);
    } else {
      for (int k = idx; k < a.n; ++k) {
        if (t >= 0)
          steady<1, false>(a, op, k, t, cf, acc);
        else
          startup<1, false>(a, op, k, a.i, cf.sigma_i, acc);
      }
    }
  }
};

}  // namespace plcg
