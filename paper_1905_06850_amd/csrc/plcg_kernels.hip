// Device code of libplcg for gfx950 (MI355X).
//
// Every kernel streams the unknowns in chunks of kChunk = 512 consecutive
// indices (two per thread, 16-byte loads).  Chunks are dealt to workgroups so
// that each of the 8 XCDs owns one contiguous band of the grid: the hardware
// hands workgroup b to XCD b % 8, so workgroup b works on band b % 8, chunk
// (b / 8) + k * (gridDim / 8).  Stencil neighbours in the next or previous row
// or plane are then read by workgroups on the same XCD and hit its L2.
//
// Reductions are deterministic: each workgroup reduces its products in a fixed
// order (per-thread sums, wave butterfly, waves in order) and stores one
// partial per dot product; the last workgroup to take the atomic ticket adds
// the partials in workgroup order and runs the O(l^2) scalar steps of the
// method in one thread, from a copy of the scalar state in LDS.
#include "plcg_internal.h"

#include <math.h>

namespace plcg {

// ---------------------------------------------------------------------------
// Chunk scheduling and stencil helpers
// ---------------------------------------------------------------------------

struct ChunkIter {
  int c, end, step;
};

__device__ inline ChunkIter xcd_chunks(int nchunks) {
  const int band = blockIdx.x % kXcds;
  const int lb = blockIdx.x / kXcds;
  const int nlb = gridDim.x / kXcds;
  const int lo = (int)(((long long)band * nchunks) / kXcds);
  const int hi = (int)(((long long)(band + 1) * nchunks) / kXcds);
  return ChunkIter{lo + lb, hi, nlb};
}

struct Grid {
  int n, nx, ny, nz;
};

// Sum of the face neighbours of unknown p (zero outside the grid).
template <bool D3>
__device__ inline double neighbour_sum(const double *z, int p, const Grid &g) {
  const int x = p % g.nx;
  const int rest = p / g.nx;
  const int y = D3 ? rest % g.ny : rest;
  double s = 0.0;
  if (x > 0) s += z[p - 1];
  if (x < g.nx - 1) s += z[p + 1];
  if (y > 0) s += z[p - g.nx];
  if (y < g.ny - 1) s += z[p + g.nx];
  if (D3) {
    const int zz = rest / g.ny;
    const int plane = g.nx * g.ny;
    if (zz > 0) s += z[p - plane];
    if (zz < g.nz - 1) s += z[p + plane];
  }
  return s;
}

template <int V>
struct Vals {
  double v[V];
  __device__ inline void load(const double *p) {
    if constexpr (V == 2) {
      const double2 t = *reinterpret_cast<const double2 *>(p);
      v[0] = t.x;
      v[1] = t.y;
    } else {
      v[0] = *p;
    }
  }
  __device__ inline void store(double *p) const {
    if constexpr (V == 2) {
      *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    } else {
      *p = v[0];
    }
  }
  __device__ inline void zero() {
#pragma unroll
    for (int k = 0; k < V; ++k) v[k] = 0.0;
  }
};

// ---------------------------------------------------------------------------
// Deterministic block reduction and the last-block ticket
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Reduce acc[0..ND-1] over the workgroup; result valid in out[] (LDS) after the call.
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

// Store this workgroup's partials, take a ticket; returns true in the last
// workgroup, which then holds the grid-wide sums in tot[] (LDS).
template <int ND>
__device__ inline bool reduce_grid(const double (&acc)[ND], double *partials, int max_blocks,
                                   int32_t *ticket, double *lds, double *blk, double *tot) {
  __shared__ int s_last;
  block_sum<ND>(acc, lds, blk);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < ND; ++m) partials[m * max_blocks + blockIdx.x] = blk[m];
    __threadfence();
    const int tk = atomicAdd(ticket, 1);
    s_last = (tk == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
  double sums[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    double s = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kThreads) s += partials[m * max_blocks + b];
    sums[m] = s;
  }
  block_sum<ND>(sums, lds, tot);
  if (threadIdx.x == 0) *ticket = 0;
  return true;
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

__device__ inline void publish(const DevState &s, HostStatus *hs, double zeta) {
  hs->status = s.status;
  hs->last_t = s.last_t;
  hs->cols = s.cols;
  hs->zeta = zeta;
  hs->beta = s.beta;
  hs->rref = s.rref;
  hs->sumsq = s.sumsq;
  __threadfence_system();
}

// ---------------------------------------------------------------------------
// Scalar engine of p(l)-CG: one column of G, one column of T, one LU step
// ---------------------------------------------------------------------------

__device__ inline double &gref(DevState &s, int r, int c) {
  return s.g[c % kGRing][r - c + 2 * kLMax];
}

__device__ inline bool finite_d(double v) { return isfinite(v); }

// Column c of G from the raw products raw[0] = (z_c, v_{c-l}) and
// raw[m] = (z_c, z_{c-l+m}), m = 1..l (Sec. 2.1 corrections, Eq. symmetry_G),
// then gamma_t, delta_t (Eqs. haa1, haa3), eta_t, zeta_t (Eq. LU) for t = c-1,
// then the breakdown and convergence tests.  Runs in one thread.
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
  bool broken = !(finite_d(arg) && arg > 0.0);
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
    broken = !(finite_d(gam) && finite_d(dlt) && dlt > 0.0);
    if (!broken) {
      if (t == 0) {
        eta = gam;
        zeta = s.beta;
      } else {
        const double lam = s.dlt[(t - 1) % kTRing] / s.eta[(t - 1) % kTRing];
        eta = gam - lam * s.dlt[(t - 1) % kTRing];
        zeta = -lam * s.zeta[(t - 1) % kTRing];
      }
      broken = !(finite_d(eta) && eta > 0.0 && finite_d(zeta));
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

template <int L, bool D3>
struct Sweep {
  static constexpr int ND = L + 1;

  // Steady state, i >= l: K1 (SpMV of z^{(l)}_i), K4 (all basis recurrences),
  // K6 (p_t, x_t), K5 (l+1 products for column i+1).
  template <int V>
  __device__ static inline void steady(const SweepArgs &a, const Grid &g, int idx, int t,
                                       double gam, double dm1, double inv_del, double inv_eta,
                                       double zm1, const double *sig, double (&acc)[ND]) {
    Vals<V> zc, zp;
    zc.load(a.zl[0] + idx);
    zp.load(a.zl[1] + idx);
    const double diag = D3 ? 6.0 : 4.0;
    double zn[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double w = diag * zc.v[v] - neighbour_sum<D3>(a.zl[0], idx + v, g);
      zn[v] = ((w - gam * zc.v[v]) - dm1 * zp.v[v]) * inv_del;
    }
    // Dot products against older z^{(l)} history, read before zl_out is written
    // (zl_out is the slot of z^{(l)}_{i+1-R}).
#pragma unroll
    for (int m = 1; m <= L - 3; ++m) {
      Vals<V> zh;
      zh.load(a.zl[L - 1 - m] + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) acc[m] += zn[v] * zh.v[v];
    }
    double above[V], vt[V], vnew[V];
#pragma unroll
    for (int v = 0; v < V; ++v) above[v] = zc.v[v];
#pragma unroll
    for (int k = L - 1; k >= 0; --k) {
      Vals<V> ck, pk;
      ck.load(a.zk_cur[k] + idx);
      if (t >= 1) pk.load(a.zk_prev[k] + idx); else pk.zero();
      Vals<V> nk;
      const double sk = sig[k] - gam;
#pragma unroll
      for (int v = 0; v < V; ++v) nk.v[v] = ((above[v] + sk * ck.v[v]) - dm1 * pk.v[v]) * inv_del;
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
    Vals<V> pv;
    if (t == 0) {
#pragma unroll
      for (int v = 0; v < V; ++v) pv.v[v] = vt[v] * inv_eta;
    } else {
      Vals<V> xv;
      pv.load(a.p + idx);
      xv.load(a.x + idx);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xv.v[v] += zm1 * pv.v[v];
        pv.v[v] = (vt[v] - dm1 * pv.v[v]) * inv_eta;
      }
      xv.store(a.x + idx);
    }
    pv.store(a.p + idx);
    Vals<V> out;
#pragma unroll
    for (int v = 0; v < V; ++v) out.v[v] = zn[v];
    out.store(a.zl_out + idx);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc[0] += zn[v] * vnew[v];            // (z_{i+1}, v_{t+1})
      acc[L] += zn[v] * zn[v];              // (z_{i+1}, z_{i+1})
      if (L >= 2) acc[L - 1] += zn[v] * zc.v[v];   // (z_{i+1}, z_i)
      if (L >= 3) acc[L - 2] += zn[v] * zp.v[v];   // (z_{i+1}, z_{i-1})
    }
  }

  // Start-up, i < l: z^{(l)}_{i+1} = (A - sigma_i) z^{(l)}_i, copy into basis
  // i+1, products (z_{i+1}, z_j), j >= 0, and (z_l, v_0) when i = l-1.
  template <int V>
  __device__ static inline void startup(const SweepArgs &a, const Grid &g, int idx, int i,
                                        double sigma_i, double (&acc)[ND]) {
    Vals<V> zc;
    zc.load(a.zl[0] + idx);
    const double diag = D3 ? 6.0 : 4.0;
    Vals<V> zn;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double w = diag * zc.v[v] - neighbour_sum<D3>(a.zl[0], idx + v, g);
      zn.v[v] = w - sigma_i * zc.v[v];
    }
#pragma unroll
    for (int m = 1; m <= L - 2; ++m) {
      const int h = L - 1 - m;
      if (h <= i) {
        Vals<V> zh;
        zh.load(a.zl[h] + idx);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[m] += zn.v[v] * zh.v[v];
      }
    }
    if (a.v0 != nullptr) {
      Vals<V> vz;
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
};

template <int L, bool D3>
__global__ __launch_bounds__(kThreads) void plcg_sweep_kernel(SweepArgs a) {
  using S = Sweep<L, D3>;
  constexpr int ND = S::ND;
  __shared__ double lds[4 * ND];
  __shared__ double blk[ND];
  __shared__ double tot[ND];
  __shared__ DevState sh;

  const DevState *st = a.st;
  const int i = a.i;
  const int t = i - L;
  const int status = st->status;
  // Sweeps past the stop no longer change anything (the solve's x is x_{last_t}).
  if (status != kRunning && t > st->last_t) return;

  const Grid g{a.n, a.nx, a.ny, a.nz};
  double acc[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) acc[m] = 0.0;

  if (t >= 0) {
    const double gam = st->gam[t % kTRing];
    const double del = st->dlt[t % kTRing];
    const double dm1 = t >= 1 ? st->dlt[(t - 1) % kTRing] : 0.0;
    const double inv_del = 1.0 / del;
    const double inv_eta = 1.0 / st->eta[t % kTRing];
    const double zm1 = t >= 1 ? st->zeta[(t - 1) % kTRing] : 0.0;
    double sig[L];
#pragma unroll
    for (int k = 0; k < L; ++k) sig[k] = st->sigma[k];
    for (ChunkIter it = xcd_chunks(a.nchunks); it.c < it.end; it.c += it.step) {
      const int idx = it.c * kChunk + threadIdx.x * kVec;
      if (idx + 1 < a.n)
        S::template steady<2>(a, g, idx, t, gam, dm1, inv_del, inv_eta, zm1, sig, acc);
      else if (idx < a.n)
        S::template steady<1>(a, g, idx, t, gam, dm1, inv_del, inv_eta, zm1, sig, acc);
    }
  } else {
    const double sigma_i = st->sigma[i];
    for (ChunkIter it = xcd_chunks(a.nchunks); it.c < it.end; it.c += it.step) {
      const int idx = it.c * kChunk + threadIdx.x * kVec;
      if (idx + 1 < a.n)
        S::template startup<2>(a, g, idx, i, sigma_i, acc);
      else if (idx < a.n)
        S::template startup<1>(a, g, idx, i, sigma_i, acc);
    }
  }

  if (!reduce_grid<ND>(acc, a.partials, a.max_blocks, a.ticket, lds, blk, tot)) return;

  // Last workgroup: finalise column i+1 of G and the scalars for t' = i.
  state_load(st, &sh);
  if (threadIdx.x == 0 && sh.status == kRunning) {
    engine_column(sh, tot, i + 1, a.hist);
    publish(sh, a.hs, fabs(sh.zeta[i % kTRing]));
  }
  state_store(&sh, a.st);
}

// ---------------------------------------------------------------------------
// Classic CG: two sweeps per iteration
// ---------------------------------------------------------------------------

// Sweep A of iteration k: p_k = r_k + beta_{k-1} p_{k-1} (p_0 = r_0), q = A p_k,
// product (p_k, q); the last workgroup forms alpha_k = (r_k, r_k) / (p_k, q).
template <bool D3>
__global__ __launch_bounds__(kThreads) void cg_sweep_a_kernel(CgArgs a) {
  __shared__ double lds[4];
  __shared__ double blk[1];
  __shared__ double tot[1];
  const DevState *st = a.st;
  if (st->status != kRunning) return;
  const bool first = a.k == 0;
  const double beta = first ? 0.0 : st->cg_beta;
  const Grid g{a.n, a.nx, a.ny, a.nz};
  const double diag = D3 ? 6.0 : 4.0;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks); it.c < it.end; it.c += it.step) {
    const int idx0 = it.c * kChunk + threadIdx.x * kVec;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= a.n) break;
      // p_k at p and at its neighbours, formed on the fly from r and p_{k-1}
      auto pk = [&](int q) { return first ? a.r[q] : a.r[q] + beta * a.p_old[q]; };
      const double pc = pk(p);
      const int x = p % g.nx;
      const int rest = p / g.nx;
      const int y = D3 ? rest % g.ny : rest;
      double s = 0.0;
      if (x > 0) s += pk(p - 1);
      if (x < g.nx - 1) s += pk(p + 1);
      if (y > 0) s += pk(p - g.nx);
      if (y < g.ny - 1) s += pk(p + g.nx);
      if (D3) {
        const int zz = rest / g.ny;
        const int plane = g.nx * g.ny;
        if (zz > 0) s += pk(p - plane);
        if (zz < g.nz - 1) s += pk(p + plane);
      }
      const double q = diag * pc - s;
      a.p_new[p] = pc;
      a.q[p] = q;
      acc[0] += pc * q;
    }
  }
  __shared__ DevState sh;
  if (!reduce_grid<1>(acc, a.partials, a.max_blocks, a.ticket, lds, blk, tot)) return;
  state_load(st, &sh);
  if (threadIdx.x == 0) {
    const double pq = tot[0];
    if (!(isfinite(pq) && pq > 0.0)) {
      sh.status = kCgBreak;
      sh.last_t = a.k;
    } else {
      sh.cg_alpha = sh.cg_rho / pq;
    }
    publish(sh, a.hs, sqrt(sh.cg_rho));
  }
  state_store(&sh, a.st);
}

// Sweep B of iteration k: x += alpha p_k, r -= alpha q, product (r, r);
// the last workgroup forms beta_k and tests ||r_{k+1}|| < tol ||r_0||.
__global__ __launch_bounds__(kThreads) void cg_sweep_b_kernel(CgArgs a) {
  __shared__ double lds[4];
  __shared__ double blk[1];
  __shared__ double tot[1];
  const DevState *st = a.st;
  if (st->status != kRunning) return;
  const double alpha = st->cg_alpha;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks); it.c < it.end; it.c += it.step) {
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
  __shared__ DevState sh;
  if (!reduce_grid<1>(acc, a.partials, a.max_blocks, a.ticket, lds, blk, tot)) return;
  state_load(st, &sh);
  if (threadIdx.x == 0) {
    const double rho = tot[0];
    const double rn = sqrt(rho);
    sh.cols = a.k + 1;
    sh.last_t = a.k + 1;
    if (!isfinite(rho)) {
      sh.status = kCgBreak;
    } else {
      sh.cg_beta = rho / sh.cg_rho;
      sh.cg_rho = rho;
      if (rn < sh.abs_tol) sh.status = kConverged;
    }
    publish(sh, a.hs, rn);
  }
  state_store(&sh, a.st);
}

// ---------------------------------------------------------------------------
// Residual, scaling, operator application, copy
// ---------------------------------------------------------------------------

template <bool D3>
__global__ __launch_bounds__(kThreads) void residual_kernel(
    const double *b, const double *x, double *r, double *partials, int32_t *ticket, DevState *st,
    HostStatus *hs, int mode, double tol, double rref_in, Grid g, int nchunks, int max_blocks) {
  __shared__ double lds[4];
  __shared__ double blk[1];
  __shared__ double tot[1];
  const double diag = D3 ? 6.0 : 4.0;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(nchunks); it.c < it.end; it.c += it.step) {
    const int idx0 = it.c * kChunk + threadIdx.x * kVec;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= g.n) break;
      const double rv = b[p] - (diag * x[p] - neighbour_sum<D3>(x, p, g));
      if (r != nullptr) r[p] = rv;
      acc[0] += rv * rv;
    }
  }
  __shared__ DevState sh;
  if (!reduce_grid<1>(acc, partials, max_blocks, ticket, lds, blk, tot)) return;
  state_load(st, &sh);
  if (threadIdx.x == 0) {
    const double ss = tot[0];
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
      if (mode == 0) {
        for (int c = 0; c < kGRing; ++c)
          for (int r2 = 0; r2 < kBand; ++r2) sh.g[c][r2] = 0.0;
        for (int k = 0; k < kTRing; ++k) sh.gam[k] = sh.dlt[k] = sh.eta[k] = sh.zeta[k] = 0.0;
        gref(sh, 0, 0) = 1.0;
      } else {
        sh.cg_rho = ss;
        sh.cg_alpha = 0.0;
        sh.cg_beta = 0.0;
      }
    }
    publish(sh, hs, sqrt(ss));
  }
  state_store(&sh, st);
}

__global__ __launch_bounds__(kThreads) void scale_kernel(const double *r, double *d0, double *d1,
                                                          double *d2, const DevState *st, int n) {
  if (st->status != kRunning) return;
  const double inv = 1.0 / st->beta;
  for (int p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads) {
    const double v = r[p] * inv;
    if (d0) d0[p] = v;
    if (d1) d1[p] = v;
    if (d2) d2[p] = v;
  }
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

template <int L>
static hipError_t launch_sweep_l(const SweepArgs &a, int blocks, hipStream_t s) {
  if (a.d3)
    hipLaunchKernelGGL((plcg_sweep_kernel<L, true>), dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((plcg_sweep_kernel<L, false>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_plcg_sweep(const SweepArgs &a, int blocks, hipStream_t s) {
  switch (a.l) {
    case 1: return launch_sweep_l<1>(a, blocks, s);
    case 2: return launch_sweep_l<2>(a, blocks, s);
    case 3: return launch_sweep_l<3>(a, blocks, s);
    case 4: return launch_sweep_l<4>(a, blocks, s);
    case 5: return launch_sweep_l<5>(a, blocks, s);
    case 6: return launch_sweep_l<6>(a, blocks, s);
    case 7: return launch_sweep_l<7>(a, blocks, s);
    case 8: return launch_sweep_l<8>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cg_sweep_a(const CgArgs &a, int blocks, hipStream_t s) {
  if (a.d3)
    hipLaunchKernelGGL((cg_sweep_a_kernel<true>), dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((cg_sweep_a_kernel<false>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg_sweep_b(const CgArgs &a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(cg_sweep_b_kernel, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_residual(const double *b, const double *x, double *r, double *partials,
                           int32_t *ticket, DevState *st, HostStatus *hs, int mode, double tol,
                           double rref_in, int n, int nx, int ny, int nz, bool d3, int nchunks,
                           int blocks, int max_blocks, hipStream_t s) {
  const Grid g{n, nx, ny, nz};
  if (d3)
    hipLaunchKernelGGL((residual_kernel<true>), dim3(blocks), dim3(kThreads), 0, s, b, x, r,
                       partials, ticket, st, hs, mode, tol, rref_in, g, nchunks, max_blocks);
  else
    hipLaunchKernelGGL((residual_kernel<false>), dim3(blocks), dim3(kThreads), 0, s, b, x, r,
                       partials, ticket, st, hs, mode, tol, rref_in, g, nchunks, max_blocks);
  return hipGetLastError();
}

hipError_t launch_scale(const double *r, double *d0, double *d1, double *d2, DevState *st, int n,
                        int blocks, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(blocks), dim3(kThreads), 0, s, r, d0, d1, d2, st, n);
  return hipGetLastError();
}

hipError_t launch_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                        int blocks, hipStream_t s) {
  const Grid g{n, nx, ny, nz};
  if (d3)
    hipLaunchKernelGGL((apply_kernel<true>), dim3(blocks), dim3(kThreads), 0, s, x, y, g);
  else
    hipLaunchKernelGGL((apply_kernel<false>), dim3(blocks), dim3(kThreads), 0, s, x, y, g);
  return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t s) {
  int64_t pairs = (n + 1) / 2;
  int64_t blocks = (pairs + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace plcg
