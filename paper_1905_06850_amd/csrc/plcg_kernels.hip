// Device code of libplcg for gfx950 (MI355X).
//
// Streaming: every kernel walks the unknowns in chunks of kChunk = 512
// consecutive indices (two per thread, 16-byte loads).  Chunks are dealt so that
// each of the 8 XCDs owns one contiguous band of the grid: the hardware hands
// workgroup b to XCD b % 8, so workgroup b works on band b % 8.  Stencil
// neighbours in the next or previous row or plane are then read by workgroups on
// the same XCD and hit its L2.
//
// Reductions: a kernel never waits for the other workgroups of the same launch.
// Each workgroup reduces its products in a fixed order (per-thread sums, wave
// butterfly, waves in order) and stores one partial per product.  The partials
// are added up by the next launch, after the kernel boundary has made them
// visible: for p(1)-CG and classic CG, whose next iteration needs the result at
// once, every workgroup adds them itself (same order, so every workgroup gets
// the same bits); for p(l)-CG with l >= 2 one extra workgroup does it while the
// others stream, and the coefficients it produces are first used l-1 launches
// later - the reduction of iteration i-1 runs during the SpMV of iteration i
// (Sec. 3.1, Alg. 2).  No fences, atomics or host round trips per iteration.
#include "plcg_internal.h"

#include <math.h>

namespace plcg {

// ---------------------------------------------------------------------------
// Chunk scheduling
// ---------------------------------------------------------------------------

struct ChunkIter {
  int c, end, step;
};

// Streaming workgroups are blockIdx.x = first .. first + nstream - 1 (first is 0
// or 1, nstream a multiple of 8); workgroup b sits on XCD b % 8 and takes band
// b % 8 of the chunks.
__device__ inline ChunkIter xcd_chunks(int nchunks, int nstream, int first) {
  const int band = blockIdx.x % kXcds;
  const int lb = (blockIdx.x - first) / kXcds;
  const int nlb = nstream / kXcds;
  const int lo = (int)(((long long)band * nchunks) / kXcds);
  const int hi = (int)(((long long)(band + 1) * nchunks) / kXcds);
  return ChunkIter{lo + lb, hi, nlb};
}

struct Grid {
  int n, nx, ny, nz;
};

// ---------------------------------------------------------------------------
// Stencil
// ---------------------------------------------------------------------------

// V consecutive values held in FP64 registers; S is the storage type in memory
// (double, or float for the FP32-stored inner solver), converted on load/store.
template <int V, typename S = double>
struct Vals {
  double v[V];
  __device__ inline void load(const S *p) {
    if constexpr (V == 2 && sizeof(S) == 8) {
      const double2 t = *reinterpret_cast<const double2 *>(p);
      v[0] = t.x;
      v[1] = t.y;
    } else if constexpr (V == 2) {
      const float2 t = *reinterpret_cast<const float2 *>(p);
      v[0] = (double)t.x;
      v[1] = (double)t.y;
    } else {
      v[0] = (double)*p;
    }
  }
  __device__ inline void store(S *p) const {
    if constexpr (V == 2 && sizeof(S) == 8) {
      *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    } else if constexpr (V == 2) {
      *reinterpret_cast<float2 *>(p) = make_float2((float)v[0], (float)v[1]);
    } else {
      *p = (S)v[0];
    }
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

// w = A z at the V unknowns starting at idx, given their values zc.
// FAST (a full chunk and an even nx): both unknowns of a thread share a row,
// x-neighbours come from the adjacent lanes (consecutive pairs), the rows and
// planes above and below are 16-byte loads.  Called by all 64 lanes together.
template <int V, bool D3, bool FAST, typename S>
__device__ inline void apply_stencil(const S *z, int idx, const Vals<V, S> &zc, const Grid &g,
                                     double (&w)[V]) {
  const double diag = D3 ? 6.0 : 4.0;
  if constexpr (FAST && V == 2) {
    const int x = idx % g.nx;
    const int rest = idx / g.nx;
    const int y = D3 ? rest % g.ny : rest;
    const int lane = threadIdx.x & 63;
    double left = __shfl_up(zc.v[1], 1, 64);     // z[idx-1] held by the previous lane
    double right = __shfl_down(zc.v[0], 1, 64);  // z[idx+2] held by the next lane
    if (lane == 0 && x > 0) left = (double)z[idx - 1];
    if (lane == 63 && x + 2 < g.nx) right = (double)z[idx + 2];
    double s0 = (x > 0 ? left : 0.0) + zc.v[1];
    double s1 = zc.v[0] + (x + 2 < g.nx ? right : 0.0);
    if (y > 0) {
      Vals<2, S> u;
      u.load(z + idx - g.nx);
      s0 += u.v[0];
      s1 += u.v[1];
    }
    if (y < g.ny - 1) {
      Vals<2, S> d;
      d.load(z + idx + g.nx);
      s0 += d.v[0];
      s1 += d.v[1];
    }
    if (D3) {
      const int zz = rest / g.ny;
      const int plane = g.nx * g.ny;
      if (zz > 0) {
        Vals<2, S> f;
        f.load(z + idx - plane);
        s0 += f.v[0];
        s1 += f.v[1];
      }
      if (zz < g.nz - 1) {
        Vals<2, S> k;
        k.load(z + idx + plane);
        s0 += k.v[0];
        s1 += k.v[1];
      }
    }
    w[0] = diag * zc.v[0] - s0;
    w[1] = diag * zc.v[1] - s1;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) w[v] = diag * zc.v[v] - neighbour_sum<D3, S>(z, idx + v, g);
  }
}

// ---------------------------------------------------------------------------
// Deterministic block reductions
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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

// Grid-wide sums of the previous launch's partials, in a fixed order.
template <int ND>
__device__ inline void sum_partials(const double *part, int nparts, int pstride, double *lds,
                                    double *out) {
  double s[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kThreads) acc += part[m * pstride + b];
    s[m] = acc;
  }
  block_sum<ND>(s, lds, out);
}

// This workgroup's partials (index = streaming workgroup number).
template <int ND>
__device__ inline void store_partials(const double (&acc)[ND], double *part, int pstride,
                                      int slot, double *lds, double *blk) {
  block_sum<ND>(acc, lds, blk);
  if (threadIdx.x < ND) part[threadIdx.x * pstride + slot] = blk[threadIdx.x];
}

// Copy the scalar state between global memory and LDS (all threads).
__device__ inline void state_load(const DevState *st, DevState *sh) {
  const double *src = reinterpret_cast<const double *>(st);
  double *dst = reinterpret_cast<double *>(sh);
  for (int k = threadIdx.x; k < (int)(sizeof(DevState) / 8); k += kThreads) dst[k] = src[k];
  __syncthreads();
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

__device__ inline double &gref(DevState &s, int r, int c) {
  return s.g[c % kGRing][r - c + 2 * kLMax];
}

// Column c of G from the raw products raw[0] = (z_c, v_{c-l}) and
// raw[m] = (z_c, z_{c-l+m}), m = 1..l: the entries below the l-th upper
// diagonal from Eq. (symmetry_G), the forward substitution for rows
// c-l+1 .. c-1 and the square root for the diagonal (Alg. 1, update of G);
// then gamma_t, delta_t (Eqs. haa1, haa3) and eta_t, zeta_t (Eq. LU and the
// recursion for zeta) for t = c-1, and the breakdown / convergence tests.
// Runs in one thread.
__device__ void engine_column(DevState &s, const double *raw, int c, double *hist) {
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

// ---------------------------------------------------------------------------
// p(l)-CG sweep: iteration i of Alg. 1
// ---------------------------------------------------------------------------

template <int L>
struct Coef {
  double gam, dm1, inv_del, inv_eta, zm1, sigma_i;
  double sig[L];
};

template <int L, bool D3, typename S>
struct Sweep {
  using Args = SweepArgsT<S>;
  static constexpr int ND = L + 1;

  // Steady state, i >= l: K1 (SpMV of z^{(l)}_i), K4 (all basis recurrences,
  // Eqs. all_z_rec2 and specific_z_rec), K6 (p_t, x_t; Eqs. pdir, x_a2) and
  // K5 (the l+1 products that start column i+1 of G).
  template <int V, bool FAST>
  __device__ static inline void steady(const Args &a, const Grid &g, int idx, int t,
                                       const Coef<L> &cf, double (&acc)[ND]) {
    Vals<V, S> zc, zp;
    zc.load(a.zl[0] + idx);
    zp.load(a.zl[1] + idx);
    double w[V];
    apply_stencil<V, D3, FAST, S>(a.zl[0], idx, zc, g, w);
    double zn[V];
#pragma unroll
    for (int v = 0; v < V; ++v) zn[v] = ((w[v] - cf.gam * zc.v[v]) - cf.dm1 * zp.v[v]) * cf.inv_del;
    // Products with older z^{(l)} vectors, read before zl_out (the slot of
    // z^{(l)}_{i+1-R}) is overwritten below.
#pragma unroll
    for (int m = 1; m <= L - 3; ++m) {
      Vals<V, S> zh;
      zh.load(a.zl[L - 1 - m] + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[m] += zn[v] * zh.v[v];
    }
    double above[V], vt[V], vnew[V];
#pragma unroll
    for (int v = 0; v < V; ++v) above[v] = zc.v[v];
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
      Vals<V, S> ck, pk;
      ck.load(a.zk_cur[k] + idx);
      if (t >= 1) pk.load(a.zk_prev[k] + idx); else pk.zero();
      Vals<V, S> nk;
      const double sk = cf.sig[k] - cf.gam;
#pragma unroll
      for (int v = 0; v < V; ++v) nk.v[v] = ((above[v] + sk * ck.v[v]) - cf.dm1 * pk.v[v]) * cf.inv_del;
      nk.store(a.zk_prev[k] + idx);
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
    } else {
      Vals<V, S> xv;
      pv.load(a.p + idx);
      xv.load(a.x + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xv.v[v] += cf.zm1 * pv.v[v];
        pv.v[v] = (vt[v] - cf.dm1 * pv.v[v]) * cf.inv_eta;
      }
      xv.store(a.x + idx);
    }
    pv.store(a.p + idx);
    Vals<V, S> out;
#pragma unroll
    for (int v = 0; v < V; ++v) out.v[v] = zn[v];
    out.store(a.zl_out + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[0] += zn[v] * vnew[v];                    // (z_{i+1}, v_{t+1})
      acc[L] += zn[v] * zn[v];                      // (z_{i+1}, z_{i+1})
      if (L >= 2) acc[L - 1] += zn[v] * zc.v[v];    // (z_{i+1}, z_i)
      if (L >= 3) acc[L - 2] += zn[v] * zp.v[v];    // (z_{i+1}, z_{i-1})
    }
  }

  // Start-up, i < l: z^{(l)}_{i+1} = (A - sigma_i) z^{(l)}_i, copied into basis
  // i+1; products (z_{i+1}, z_j), j >= 0, and (z_l, v_0) when i = l-1.
  template <int V, bool FAST>
  __device__ static inline void startup(const Args &a, const Grid &g, int idx, int i,
                                        double sigma_i, double (&acc)[ND]) {
    Vals<V, S> zc;
    zc.load(a.zl[0] + idx);
    double w[V];
    apply_stencil<V, D3, FAST, S>(a.zl[0], idx, zc, g, w);
    Vals<V, S> zn;
#pragma unroll
    for (int v = 0; v < V; ++v) zn.v[v] = w[v] - sigma_i * zc.v[v];
#pragma unroll
    for (int m = 1; m <= L - 2; ++m) {
      const int h = L - 1 - m;
      if (h <= i) {
        Vals<V, S> zh;
        zh.load(a.zl[h] + idx);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[m] += zn.v[v] * zh.v[v];
      }
    }
    if (a.v0 != nullptr) {
      Vals<V, S> vz;
      vz.load(a.v0 + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[0] += zn.v[v] * vz.v[v];
    }
    zn.store(a.zl_out + idx);
    if (a.copy_dst != nullptr) zn.store(a.copy_dst + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[L] += zn.v[v] * zn.v[v];
      if (L >= 2) acc[L - 1] += zn.v[v] * zc.v[v];
    }
  }

  template <bool FAST>
  __device__ static inline void chunk(const Args &a, const Grid &g, int idx, int t,
                                      const Coef<L> &cf, double (&acc)[ND]) {
    if (t >= 0) {
      if (idx + 1 < a.n)
        steady<2, FAST>(a, g, idx, t, cf, acc);
      else if (idx < a.n)
        steady<1, false>(a, g, idx, t, cf, acc);
    } else {
      if (idx + 1 < a.n)
        startup<2, FAST>(a, g, idx, a.i, cf.sigma_i, acc);
      else if (idx < a.n)
        startup<1, false>(a, g, idx, a.i, cf.sigma_i, acc);
    }
  }
};

template <int L>
__device__ inline void read_coef(const DevState &s, int i, int t, Coef<L> &cf) {
  if (t >= 0) {
    cf.gam = s.gam[t % kTRing];
    cf.inv_del = 1.0 / s.dlt[t % kTRing];
    cf.dm1 = t >= 1 ? s.dlt[(t - 1) % kTRing] : 0.0;
    cf.inv_eta = 1.0 / s.eta[t % kTRing];
    cf.zm1 = t >= 1 ? s.zeta[(t - 1) % kTRing] : 0.0;
    cf.sigma_i = 0.0;
  } else {
    cf.gam = cf.inv_del = cf.dm1 = cf.inv_eta = cf.zm1 = 0.0;
    cf.sigma_i = s.sigma[i];
  }
#pragma unroll
  for (int k = 0; k < L; ++k) cf.sig[k] = s.sigma[k];
}

template <int L, bool D3, typename ST>
__global__ __launch_bounds__(kThreads) void plcg_sweep_kernel(SweepArgsT<ST> a) {
  using S = Sweep<L, D3, ST>;
  constexpr int ND = S::ND;
  __shared__ double lds[4 * ND];
  __shared__ double red[ND];
  __shared__ DevState sh;

  // Workgroup 0 owns the scalar state and carries it from launch i-1 to launch
  // i.  For l = 1 every workgroup finalises column i itself (this launch needs
  // it); for l >= 2 only workgroup 0 does, and it streams nothing.
  const bool owner = blockIdx.x == 0;
  const bool engine = (L == 1) || owner;
  if (engine) {
    state_load(a.st_in, &sh);
    if (a.i >= 1 && sh.status == kRunning && a.nparts_in > 0) {
      sum_partials<ND>(a.part_in, a.nparts_in, a.pstride, lds, red);
      if (threadIdx.x == 0) engine_column(sh, red, a.i, owner ? a.hist : nullptr);
      __syncthreads();
    }
    if (owner) {
      state_store(&sh, a.st_out);
      if (threadIdx.x == 0) publish(sh, a.hs, fabs(sh.zeta[(a.i + kTRing - 1) % kTRing]), a.i);
    }
    if (L >= 2) return;
  }
  if (!a.work) return;

  const int i = a.i;
  const int t = i - L;
  int status, last_t;
  Coef<L> cf;
  if (L == 1) {
    status = sh.status;
    last_t = sh.last_t;
    read_coef<L>(sh, i, t, cf);
  } else {
    status = a.st_in->status;
    last_t = a.st_in->last_t;
    read_coef<L>(*a.st_in, i, t, cf);
  }
  // Sweeps past the stop change nothing (the solve's x is x_{last_t}).
  if (status != kRunning && t > last_t) return;

  const Grid g{a.n, a.nx, a.ny, a.nz};
  double acc[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) acc[m] = 0.0;
  const int first = L == 1 ? 0 : 1;
  const bool fast_rows = (a.nx & 1) == 0;
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, first); it.c < it.end; it.c += it.step) {
    const int base = it.c * kChunk;
    const int idx = base + threadIdx.x * kVec;
    if (fast_rows && base + kChunk <= a.n)
      S::template chunk<true>(a, g, idx, t, cf, acc);
    else
      S::template chunk<false>(a, g, idx, t, cf, acc);
  }
  store_partials<ND>(acc, a.part_out, a.pstride, blockIdx.x - first, lds, red);
}

// ---------------------------------------------------------------------------
// Classic CG: two sweeps per iteration
// ---------------------------------------------------------------------------

// Sweep A of iteration k.  Prologue (every workgroup): rho_k = (r_k, r_k) from
// sweep B of iteration k-1, beta_{k-1} = rho_k / rho_{k-1}, stopping test
// ||r_k|| < tol ||r_0||.  Then p_k = r_k + beta_{k-1} p_{k-1} (p_0 = r_0),
// q = A p_k and the product (p_k, q).
template <bool D3>
__global__ __launch_bounds__(kThreads) void cg_sweep_a_kernel(CgArgs a) {
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  state_load(a.st_in, &sh);
  if (a.k >= 1 && sh.status == kRunning) {
    sum_partials<1>(a.part_in, a.nparts_in, a.pstride, lds, red);
    if (threadIdx.x == 0) {
      const double rho = red[0];
      sh.cols = a.k;
      sh.last_t = a.k;
      if (!isfinite(rho)) {
        sh.status = kCgBreak;
      } else {
        sh.cg_beta = rho / sh.cg_rho;
        sh.cg_rho = rho;
        if (sqrt(rho) < sh.abs_tol) sh.status = kConverged;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    state_store(&sh, a.st_out);
    if (threadIdx.x == 0) publish(sh, a.hs, sqrt(sh.cg_rho), 2 * a.k);
  }
  if (sh.status != kRunning || !a.work) return;

  const bool first = a.k == 0;
  const double beta = first ? 0.0 : sh.cg_beta;
  const Grid g{a.n, a.nx, a.ny, a.nz};
  const double diag = D3 ? 6.0 : 4.0;
  const bool fast_rows = (a.nx & 1) == 0;
  double acc[1] = {0.0};
  // p_k at index q, formed on the fly from r and p_{k-1}
  auto pk1 = [&](int q) { return first ? a.r[q] : a.r[q] + beta * a.p_old[q]; };
  auto pk2 = [&](int q, double &v0, double &v1) {
    Vals<2> rr;
    rr.load(a.r + q);
    v0 = rr.v[0];
    v1 = rr.v[1];
    if (!first) {
      Vals<2> po;
      po.load(a.p_old + q);
      v0 += beta * po.v[0];
      v1 += beta * po.v[1];
    }
  };
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int base = it.c * kChunk;
    const int idx0 = base + threadIdx.x * kVec;
    if (fast_rows && base + kChunk <= a.n) {
      // Same layout as the p(l)-CG fast path: pairs in one row, x-neighbours
      // from the adjacent lanes, 16-byte loads for the other rows and planes.
      double c0, c1;
      pk2(idx0, c0, c1);
      const int x = idx0 % g.nx;
      const int rest = idx0 / g.nx;
      const int y = D3 ? rest % g.ny : rest;
      const int lane = threadIdx.x & 63;
      double left = __shfl_up(c1, 1, 64);
      double right = __shfl_down(c0, 1, 64);
      if (lane == 0 && x > 0) left = pk1(idx0 - 1);
      if (lane == 63 && x + 2 < g.nx) right = pk1(idx0 + 2);
      double s0 = (x > 0 ? left : 0.0) + c1;
      double s1 = c0 + (x + 2 < g.nx ? right : 0.0);
      double u0, u1;
      if (y > 0) {
        pk2(idx0 - g.nx, u0, u1);
        s0 += u0;
        s1 += u1;
      }
      if (y < g.ny - 1) {
        pk2(idx0 + g.nx, u0, u1);
        s0 += u0;
        s1 += u1;
      }
      if (D3) {
        const int zz = rest / g.ny;
        const int plane = g.nx * g.ny;
        if (zz > 0) {
          pk2(idx0 - plane, u0, u1);
          s0 += u0;
          s1 += u1;
        }
        if (zz < g.nz - 1) {
          pk2(idx0 + plane, u0, u1);
          s0 += u0;
          s1 += u1;
        }
      }
      Vals<2> pn, qv;
      pn.v[0] = c0;
      pn.v[1] = c1;
      qv.v[0] = diag * c0 - s0;
      qv.v[1] = diag * c1 - s1;
      pn.store(a.p_new + idx0);
      qv.store(a.q + idx0);
      acc[0] += c0 * qv.v[0] + c1 * qv.v[1];
      continue;
    }
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= a.n) break;
      const double pc = pk1(p);
      const int x = p % g.nx;
      const int rest = p / g.nx;
      const int y = D3 ? rest % g.ny : rest;
      double s = 0.0;
      if (x > 0) s += pk1(p - 1);
      if (x < g.nx - 1) s += pk1(p + 1);
      if (y > 0) s += pk1(p - g.nx);
      if (y < g.ny - 1) s += pk1(p + g.nx);
      if (D3) {
        const int zz = rest / g.ny;
        const int plane = g.nx * g.ny;
        if (zz > 0) s += pk1(p - plane);
        if (zz < g.nz - 1) s += pk1(p + plane);
      }
      const double q = diag * pc - s;
      a.p_new[p] = pc;
      a.q[p] = q;
      acc[0] += pc * q;
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// Sweep B of iteration k.  Prologue: alpha_k = rho_k / (p_k, q) from sweep A
// (breakdown if (p_k, A p_k) <= 0).  Then x += alpha p_k, r -= alpha q and the
// product (r_{k+1}, r_{k+1}).
__global__ __launch_bounds__(kThreads) void cg_sweep_b_kernel(CgArgs a) {
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  state_load(a.st_in, &sh);
  if (sh.status == kRunning) {
    sum_partials<1>(a.part_in, a.nparts_in, a.pstride, lds, red);
    if (threadIdx.x == 0) {
      const double pq = red[0];
      if (!(isfinite(pq) && pq > 0.0)) {
        sh.status = kCgBreak;
        sh.last_t = a.k;
      } else {
        sh.cg_alpha = sh.cg_rho / pq;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0) {
    state_store(&sh, a.st_out);
    if (threadIdx.x == 0) publish(sh, a.hs, sqrt(sh.cg_rho), 2 * a.k + 1);
  }
  if (sh.status != kRunning || !a.work) return;

  const double alpha = sh.cg_alpha;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx = it.c * kChunk + threadIdx.x * kVec;
    if (idx + 1 < a.n) {
      Vals<2> x, p, r, q;
      x.load(a.x + idx);
      p.load(a.p_new + idx);
      r.load(a.r + idx);
      q.load(a.q + idx);
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        x.v[v] += alpha * p.v[v];
        r.v[v] -= alpha * q.v[v];
        acc[0] += r.v[v] * r.v[v];
      }
      x.store(a.x + idx);
      r.store(a.r + idx);
    } else if (idx < a.n) {
      a.x[idx] += alpha * a.p_new[idx];
      const double rv = a.r[idx] - alpha * a.q[idx];
      a.r[idx] = rv;
      acc[0] += rv * rv;
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// ---------------------------------------------------------------------------
// Residual, segment start, scaling, operator application, copy
// ---------------------------------------------------------------------------

template <bool D3>
__global__ __launch_bounds__(kThreads) void residual_kernel(const double *b, const double *x,
                                                            double *r, double *part_out, Grid g,
                                                            int nchunks, int nstream) {
  __shared__ double lds[4];
  __shared__ double red[1];
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(nchunks, nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx0 = it.c * kChunk + threadIdx.x * kVec;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= g.n) break;
      const double rv = b[p] - ((D3 ? 6.0 : 4.0) * x[p] - neighbour_sum<D3>(x, p, g));
      if (r != nullptr) r[p] = rv;
      acc[0] += rv * rv;
    }
  }
  store_partials<1>(acc, part_out, kMaxStream, blockIdx.x, lds, red);
}

// One workgroup: ||b - A x||^2 from the residual partials; starts a segment.
__global__ __launch_bounds__(kThreads) void start_kernel(const double *part_in, int nparts,
                                                         DevState *st, HostStatus *hs, int mode,
                                                         double tol, double rref_in) {
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  state_load(st, &sh);
  sum_partials<1>(part_in, nparts, kMaxStream, lds, red);
  if (threadIdx.x == 0) {
    const double ss = red[0];
    sh.sumsq = ss;
    if (mode != 2) {
      const double beta = sqrt(ss);
      sh.beta = beta;
      sh.rref = rref_in > 0.0 ? rref_in : beta;
      sh.abs_tol = tol * sh.rref;
      sh.cols = 0;
      sh.last_t = 0;
      if (!isfinite(beta)) {
        sh.status = kNonFinite;
      } else if (beta == 0.0 || beta < sh.abs_tol) {
        sh.status = kConverged;
      } else {
        sh.status = kRunning;
        sh.last_t = -1;
      }
      for (int c = 0; c < kGRing; ++c)
        for (int r2 = 0; r2 < kBand; ++r2) sh.g[c][r2] = 0.0;
      for (int k = 0; k < kTRing; ++k) sh.gam[k] = sh.dlt[k] = sh.eta[k] = sh.zeta[k] = 0.0;
      gref(sh, 0, 0) = 1.0;                    // g_00 = 1 (Alg. 1, first line)
      sh.cg_rho = ss;
      sh.cg_alpha = 0.0;
      sh.cg_beta = 0.0;
    }
    publish(sh, hs, sqrt(ss), -1);
  }
  state_store(&sh, st);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scale_kernel(const double *r, T *d0, T *d1, T *d2,
                                                          const DevState *st, int n) {
  if (st->status != kRunning) return;
  const double inv = 1.0 / st->beta;
  for (int p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads) {
    const T v = (T)(r[p] * inv);
    if (d0) d0[p] = v;
    if (d1) d1[p] = v;
    if (d2) d2[p] = v;
  }
}

// x += d: the FP32 correction of one refinement step added to the FP64 iterate.
__global__ __launch_bounds__(kThreads) void add_correction_kernel(double *x, const float *d, int n) {
  for (int p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads)
    x[p] += (double)d[p];
}

template <bool D3>
__global__ __launch_bounds__(kThreads) void apply_kernel(const double *x, double *y, Grid g) {
  const double diag = D3 ? 6.0 : 4.0;
  for (int p = blockIdx.x * kThreads + threadIdx.x; p < g.n; p += gridDim.x * kThreads)
    y[p] = diag * x[p] - neighbour_sum<D3>(x, p, g);
}

__global__ __launch_bounds__(kThreads) void copy_kernel(const double *src, double *dst, int64_t n) {
  const int64_t pairs = n / 2;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x; k < pairs; k += stride)
    reinterpret_cast<double2 *>(dst)[k] = reinterpret_cast<const double2 *>(src)[k];
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static int simple_blocks(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

template <int L, typename S>
static hipError_t launch_sweep_l(const SweepArgsT<S> &a, hipStream_t s) {
  const int grid = a.nstream + (L >= 2 ? 1 : 0);
  if (a.d3)
    hipLaunchKernelGGL((plcg_sweep_kernel<L, true, S>), dim3(grid), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((plcg_sweep_kernel<L, false, S>), dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename S>
static hipError_t launch_sweep_any(const SweepArgsT<S> &a, hipStream_t s) {
  switch (a.l) {
    case 1: return launch_sweep_l<1, S>(a, s);
    case 2: return launch_sweep_l<2, S>(a, s);
    case 3: return launch_sweep_l<3, S>(a, s);
    case 4: return launch_sweep_l<4, S>(a, s);
    case 5: return launch_sweep_l<5, S>(a, s);
    case 6: return launch_sweep_l<6, S>(a, s);
    case 7: return launch_sweep_l<7, S>(a, s);
    case 8: return launch_sweep_l<8, S>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plcg_sweep(const SweepArgsT<double> &a, hipStream_t s) {
  return launch_sweep_any<double>(a, s);
}

hipError_t launch_plcg_sweep(const SweepArgsT<float> &a, hipStream_t s) {
  return launch_sweep_any<float>(a, s);
}

hipError_t launch_cg_sweep_a(const CgArgs &a, hipStream_t s) {
  if (a.d3)
    hipLaunchKernelGGL((cg_sweep_a_kernel<true>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((cg_sweep_a_kernel<false>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg_sweep_b(const CgArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(cg_sweep_b_kernel, dim3(a.nstream), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_residual(const double *b, const double *x, double *r, double *part_out, int n,
                           int nx, int ny, int nz, bool d3, int nchunks, int nstream,
                           hipStream_t s) {
  const Grid g{n, nx, ny, nz};
  if (d3)
    hipLaunchKernelGGL((residual_kernel<true>), dim3(nstream), dim3(kThreads), 0, s, b, x, r,
                       part_out, g, nchunks, nstream);
  else
    hipLaunchKernelGGL((residual_kernel<false>), dim3(nstream), dim3(kThreads), 0, s, b, x, r,
                       part_out, g, nchunks, nstream);
  return hipGetLastError();
}

hipError_t launch_start(const double *part_in, int nparts, DevState *st, HostStatus *hs, int mode,
                        double tol, double rref_in, hipStream_t s) {
  hipLaunchKernelGGL(start_kernel, dim3(1), dim3(kThreads), 0, s, part_in, nparts, st, hs, mode,
                     tol, rref_in);
  return hipGetLastError();
}

hipError_t launch_scale(const double *r, double *d0, double *d1, double *d2, const DevState *st,
                        int n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<double>, dim3(simple_blocks(n)), dim3(kThreads), 0, s, r, d0, d1,
                     d2, st, n);
  return hipGetLastError();
}

hipError_t launch_scale(const double *r, float *d0, float *d1, float *d2, const DevState *st, int n,
                        hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<float>, dim3(simple_blocks(n)), dim3(kThreads), 0, s, r, d0, d1,
                     d2, st, n);
  return hipGetLastError();
}

hipError_t launch_add_correction(double *x, const float *d, int n, hipStream_t s) {
  hipLaunchKernelGGL(add_correction_kernel, dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, d, n);
  return hipGetLastError();
}

hipError_t launch_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                        hipStream_t s) {
  const Grid g{n, nx, ny, nz};
  if (d3)
    hipLaunchKernelGGL((apply_kernel<true>), dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, y, g);
  else
    hipLaunchKernelGGL((apply_kernel<false>), dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, y, g);
  return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(simple_blocks((n + 1) / 2)), dim3(kThreads), 0, s, src, dst,
                     n);
  return hipGetLastError();
}

}  // namespace plcg
