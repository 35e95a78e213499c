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
// Each workgroup reduces its products in a fixed order (per-thread sums,
// wave_sum, waves in order) and stores one partial per product.  The partials
// are added up by the next launch, after the kernel boundary has made them
// visible: for p(1)-CG and classic CG, whose next iteration needs the result at
// once, every workgroup adds them itself (same order, so every workgroup gets
// the same bits); for p(l)-CG with l >= 2 one extra workgroup does it while the
// others stream, and the coefficients it produces are first used l-1 launches
// later - the reduction of iteration i-1 runs during the SpMV of iteration i
// (Sec. 3.1, Alg. 2).  No fences, atomics or host round trips per iteration.
#include "plcg_sweep.h"

namespace plcg {

// ---------------------------------------------------------------------------
// p(l)-CG sweep: iteration i of Alg. 1
// ---------------------------------------------------------------------------

// P: paired x updates (Sweep's PAIR).
template <int L, bool D3, typename ST, int H, bool P>
__global__ __launch_bounds__(kThreads) void plcg_sweep_kernel(SweepArgsT<ST> a) {
  const Grid g{a.n, a.nx, a.ny, a.nz};
  plcg_sweep<L, ST, H, P>(a, ConstOp<D3, ST>{g}, a.nx % vec_of<ST>() == 0,
                          chunk_order(g, D3, kThreads * vec_of<ST>()));
}

template <int L, typename ST, int H, bool P>
__global__ __launch_bounds__(kThreads) void plcg_diag_sweep_kernel(SweepArgsT<ST> a) {
  plcg_sweep<L, ST, H, P>(a, DiagOp<ST>{a.od.dg}, true, ChunkOrder{0, 0, 0});
}

template <int L, typename ST, int H, bool P>
__global__ __launch_bounds__(kThreads) void plcg_csr_sweep_kernel(SweepArgsT<ST> a) {
  plcg_sweep<L, ST, H, P>(
      a, CsrOp<ST, (H & kHintLoads) != 0>{a.od.rp, a.od.ci, a.od.va, a.od.ell_k, a.od.ell_ld},
      true, ChunkOrder{0, 0, 0});
}

// ---------------------------------------------------------------------------
// Classic CG: two sweeps per iteration
// ---------------------------------------------------------------------------

// p_k = r_k + beta_{k-1} p_{k-1} for a pair (p_0 = r_0), one rounding each.
__device__ inline void cg_form(bool first, double beta, const Vals<2> &r, const Vals<2> &po,
                               double &v0, double &v1) {
  v0 = r.v[0];
  v1 = r.v[1];
  if (!first) {
    v0 = fma(beta, po.v[0], v0);
    v1 = fma(beta, po.v[1], v1);
  }
}

// The raw r and p_{k-1} values the fast path of sweep A reads for the pair
// idx, idx+1 (x even): its own, the rows above and below (halo), and the
// x-neighbour at the wave's edge (lane 0: x-1, lane 63: x+2).  p_{k-1} is not
// read at k = 0.
struct CgRaw {
  Vals<2> r, p, ur, up, dr, dp;
  double er, ep;
};

__device__ inline void cg_raw_fetch(const CgArgs &a, bool first, const Grid &g, int idx, int x,
                                    int y, bool halo, CgRaw &w) {
  const int lane = threadIdx.x & 63;
  w.r.load(a.r + idx);
  if (!first) w.p.load(a.p_old + idx);
  if (!halo) return;
  if (y > 0) {
    w.ur.load(a.r + idx - g.nx);
    if (!first) w.up.load(a.p_old + idx - g.nx);
  }
  if (y < g.ny - 1) {
    w.dr.load(a.r + idx + g.nx);
    if (!first) w.dp.load(a.p_old + idx + g.nx);
  }
  const int e = lane == 0 ? idx - 1 : idx + 2;
  if ((lane == 0 && x > 0) || (lane == 63 && x + 2 < g.nx)) {
    w.er = a.r[e];
    if (!first) w.ep = a.p_old[e];
  }
}

// Where the fast path gets p_k around its pair idx0, idx0+1: formed from r and
// p_{k-1} loaded where used (the loop's chunks) ...
struct CgFromMemory {
  const double *r, *po;
  double beta;
  bool first;
  int idx0, nx, plane;
  __device__ inline void pair(int q, double &v0, double &v1) const {
    Vals<2> rr, pp;
    rr.load(r + q);
    if (!first) pp.load(po + q);
    cg_form(first, beta, rr, pp, v0, v1);
  }
  __device__ inline double one(int q) const { return first ? r[q] : fma(beta, po[q], r[q]); }
  __device__ inline void own(double &v0, double &v1) const { pair(idx0, v0, v1); }
  __device__ inline double left() const { return one(idx0 - 1); }
  __device__ inline double right() const { return one(idx0 + 2); }
  __device__ inline void up(double &v0, double &v1) const { pair(idx0 - nx, v0, v1); }
  __device__ inline void down(double &v0, double &v1) const { pair(idx0 + nx, v0, v1); }
  __device__ inline void front(double &v0, double &v1) const { pair(idx0 - plane, v0, v1); }
  __device__ inline void back(double &v0, double &v1) const { pair(idx0 + plane, v0, v1); }
};

// ... or from raw values loaded ahead (a 2D sweep's first chunk).  The same
// roundings either way.
struct CgFromRaw {
  const CgRaw &w;
  double beta;
  bool first;
  __device__ inline void own(double &v0, double &v1) const { cg_form(first, beta, w.r, w.p, v0, v1); }
  __device__ inline double left() const { return first ? w.er : fma(beta, w.ep, w.er); }
  __device__ inline double right() const { return left(); }
  __device__ inline void up(double &v0, double &v1) const { cg_form(first, beta, w.ur, w.up, v0, v1); }
  __device__ inline void down(double &v0, double &v1) const { cg_form(first, beta, w.dr, w.dp, v0, v1); }
};

// Fast path of sweep A for one pair of a full chunk (nx even: the pair shares a
// row): p_k, q = A p_k and (p_k, q), x-neighbours from the adjacent lanes, the
// wave's edges, rows and planes from src.
template <bool D3, bool NTS, typename Src>
__device__ inline void cg_a_fast(const CgArgs &a, const Grid &g, int idx0, const Src &src,
                                 double (&acc)[1]) {
  const double diag = D3 ? 6.0 : 4.0;
  double c0, c1;
  src.own(c0, c1);
  const int x = idx0 % g.nx;
  const int rest = idx0 / g.nx;
  const int y = D3 ? rest % g.ny : rest;
  const int lane = threadIdx.x & 63;
  double left = lane_prev(c1);
  double right = lane_next(c0);
  if (lane == 0 && x > 0) left = src.left();
  if (lane == 63 && x + 2 < g.nx) right = src.right();
  double s0 = (x > 0 ? left : 0.0) + c1;
  double s1 = c0 + (x + 2 < g.nx ? right : 0.0);
  double u0, u1;
  if (y > 0) {
    src.up(u0, u1);
    s0 += u0;
    s1 += u1;
  }
  if (y < g.ny - 1) {
    src.down(u0, u1);
    s0 += u0;
    s1 += u1;
  }
  if constexpr (D3) {
    const int zz = rest / g.ny;
    if (zz > 0) {
      src.front(u0, u1);
      s0 += u0;
      s1 += u1;
    }
    if (zz < g.nz - 1) {
      src.back(u0, u1);
      s0 += u0;
      s1 += u1;
    }
  }
  Vals<2> pn, qv;
  pn.v[0] = c0;
  pn.v[1] = c1;
  qv.v[0] = fma(diag, c0, -s0);
  qv.v[1] = fma(diag, c1, -s1);
  pn.template st<NTS>(a.p_new + idx0);
  qv.template st<NTS>(a.q + idx0);
  acc[0] = fma(c1, qv.v[1], fma(c0, qv.v[0], acc[0]));
}

template <bool D3, int H>
__global__ __launch_bounds__(kThreads) void cg_sweep_a_kernel(CgArgs a) {
  constexpr bool NTS = (H & kHintStores) != 0;
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  const bool first = a.k == 0;
  const Grid g{a.n, a.nx, a.ny, a.nz};
  const bool fast_rows = (a.nx & 1) == 0;
  const ChunkOrder order = chunk_order(g, D3, kChunk);
  CgPrologue pro;
  cg_a_fetch(a, pro);
  // A 2D sweep then requests its first chunk's r and p_{k-1} (the pair, the
  // rows above and below, the wave-edge neighbour) before it waits for the
  // state, as the p(l)-CG sweeps do; not where vectors are stored
  // non-temporally (vectors of 96 MiB and more).
  CgRaw pre;
  bool have_pre = false;
  if constexpr (!D3 && (H & kHintStores) == 0) {
    if (a.work) {
      const ChunkIter it0 = xcd_chunks(a.nchunks, a.nstream, 0);
      if (it0.c < it0.end) {
        const int base = order.phys(it0.c) * kChunk;
        if (fast_rows && base + kChunk <= a.n) {
          const int idx0 = base + threadIdx.x * kVec;
          cg_raw_fetch(a, first, g, idx0, idx0 % g.nx, idx0 / g.nx, true, pre);
          have_pre = true;
        }
      }
    }
  }
  if (!cg_a_finish(a, pro, sh, lds, red)) return;

  const double beta = first ? 0.0 : sh.cg_beta;
  const double diag = D3 ? 6.0 : 4.0;
  double acc[1] = {0.0};
  // p_k at index q, formed on the fly from r and p_{k-1}
  auto pk1 = [&](int q) { return first ? a.r[q] : fma(beta, a.p_old[q], a.r[q]); };
  auto pk2 = [&](int q, double &v0, double &v1) {
    Vals<2> rr;
    rr.load(a.r + q);
    v0 = rr.v[0];
    v1 = rr.v[1];
    if (!first) {
      Vals<2> po;
      po.load(a.p_old + q);
      v0 = fma(beta, po.v[0], v0);
      v1 = fma(beta, po.v[1], v1);
    }
  };
  if (D3 && a.zseg > 0) {
    // z-march (3D, planes of whole chunks, even nx): a workgroup takes one
    // chunk-sized tile of a plane through zseg consecutive planes and keeps p_k
    // of the planes below, at and above the current one in registers, so every
    // r and p_{k-1} value is loaded once per plane it is the centre of (the
    // rows above and below come from the tile's own or its neighbours' loads in
    // L2).  The raw r and p_{k-1} values a plane needs (its own, the rows above
    // and below, the x-neighbours at the wave's edges) are loaded one plane
    // ahead, so their latency overlaps the current plane's work; p_k is formed
    // where it is used.  Same neighbour-sum order as the chunk path below.
    const int plane = g.nx * g.ny;
    const int ntiles = plane / kChunk;
    const int nitems = ntiles * ((g.nz + a.zseg - 1) / a.zseg);
    const int lane = threadIdx.x & 63;
    // raw loads of one plane (the plane above a segment: only its own values)
    using Raw = CgRaw;
    auto fetch = [&](int idx, int x, int y, bool halo, Raw &w) {
      cg_raw_fetch(a, first, g, idx, x, y, halo, w);
    };
    auto form = [&](const Vals<2> &r, const Vals<2> &po, double &v0, double &v1) {
      cg_form(first, beta, r, po, v0, v1);
    };
    for (ChunkIter it = xcd_chunks(nitems, a.nstream, 0); it.c < it.end; it.c += it.step) {
      const int seg = it.c / ntiles;
      const int off = (it.c - seg * ntiles) * kChunk + threadIdx.x * kVec;   // in the plane
      const int x = off % g.nx;
      const int y = off / g.nx;
      const int z0 = seg * a.zseg;
      const int z1 = min(g.nz, z0 + a.zseg);
      double m0 = 0.0, m1 = 0.0;
      if (z0 > 0) pk2(off + (z0 - 1) * plane, m0, m1);
      Raw cur, nxt;
      fetch(off + z0 * plane, x, y, true, cur);
      for (int zz = z0; zz < z1; ++zz) {
        const int idx0 = off + zz * plane;
        if (zz + 1 < g.nz) fetch(idx0 + plane, x, y, zz + 1 < z1, nxt);
        double c0, c1, n0 = 0.0, n1 = 0.0;
        form(cur.r, cur.p, c0, c1);
        if (zz + 1 < g.nz) form(nxt.r, nxt.p, n0, n1);
        double left = lane_prev(c1);
        double right = lane_next(c0);
        if (lane == 0 && x > 0) left = first ? cur.er : fma(beta, cur.ep, cur.er);
        if (lane == 63 && x + 2 < g.nx) right = first ? cur.er : fma(beta, cur.ep, cur.er);
        double s0 = (x > 0 ? left : 0.0) + c1;
        double s1 = c0 + (x + 2 < g.nx ? right : 0.0);
        double u0, u1;
        if (y > 0) {
          form(cur.ur, cur.up, u0, u1);
          s0 += u0;
          s1 += u1;
        }
        if (y < g.ny - 1) {
          form(cur.dr, cur.dp, u0, u1);
          s0 += u0;
          s1 += u1;
        }
        if (zz > 0) {
          s0 += m0;
          s1 += m1;
        }
        if (zz < g.nz - 1) {
          s0 += n0;
          s1 += n1;
        }
        Vals<2> pn, qv;
        pn.v[0] = c0;
        pn.v[1] = c1;
        qv.v[0] = fma(diag, c0, -s0);
        qv.v[1] = fma(diag, c1, -s1);
        pn.template st<NTS>(a.p_new + idx0);
        qv.template st<NTS>(a.q + idx0);
        acc[0] = fma(c1, qv.v[1], fma(c0, qv.v[0], acc[0]));
        m0 = c0;
        m1 = c1;
        cur = nxt;
      }
    }
    store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
    return;
  }
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int base = order.phys(it.c) * kChunk;
    const int idx0 = base + threadIdx.x * kVec;
    if (fast_rows && base + kChunk <= a.n) {
      // Same layout as the p(l)-CG fast path: pairs in one row, x-neighbours
      // from the adjacent lanes, 16-byte loads for the other rows and planes.
      if constexpr (!D3) {
        if (have_pre) {   // the first chunk, preloaded
          have_pre = false;
          cg_a_fast<false, NTS>(a, g, idx0, CgFromRaw{pre, beta, first}, acc);
          continue;
        }
      }
      cg_a_fast<D3, NTS>(a, g, idx0,
                         CgFromMemory{a.r, a.p_old, beta, first, idx0, g.nx, g.nx * g.ny}, acc);
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
      const double q = fma(diag, pc, -s);
      a.p_new[p] = pc;
      a.q[p] = q;
      acc[0] = fma(pc, q, acc[0]);
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// Sweep A for the diagonal operator: q = d * p_k.
template <int H>
__global__ __launch_bounds__(kThreads) void cg_diag_sweep_a_kernel(CgArgs a) {
  constexpr bool NTL = (H & kHintLoads) != 0;
  constexpr bool NTS = (H & kHintStores) != 0;
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  if (!cg_a_prologue(a, sh, lds, red)) return;

  const bool first = a.k == 0;
  const double beta = first ? 0.0 : sh.cg_beta;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx = it.c * kChunk + threadIdx.x * kVec;
    if (idx + 1 < a.n) {
      Vals<2> r, d, pn, q;
      r.template ld<NTL>(a.r + idx);
      d.template ld<NTL>(a.od.dg + idx);
      if (first) {
        pn = r;
      } else {
        Vals<2> po;
        po.template ld<NTL>(a.p_old + idx);
#pragma unroll
        for (int v = 0; v < 2; ++v) pn.v[v] = fma(beta, po.v[v], r.v[v]);
      }
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        q.v[v] = d.v[v] * pn.v[v];
        acc[0] = fma(pn.v[v], q.v[v], acc[0]);
      }
      pn.template st<NTS>(a.p_new + idx);
      q.template st<NTS>(a.q + idx);
    } else if (idx < a.n) {
      const double pc = first ? a.r[idx] : fma(beta, a.p_old[idx], a.r[idx]);
      const double q = a.od.dg[idx] * pc;
      a.p_new[idx] = pc;
      a.q[idx] = q;
      acc[0] = fma(pc, q, acc[0]);
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// Sweep A for a CSR operator: q = A p_k with p_k formed at every column index
// from r and p_{k-1}.
template <int H>
__global__ __launch_bounds__(kThreads) void cg_csr_sweep_a_kernel(CgArgs a) {
  constexpr bool NTL = (H & kHintLoads) != 0;
  constexpr bool NTS = (H & kHintStores) != 0;
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  if (!cg_a_prologue(a, sh, lds, red)) return;

  const bool first = a.k == 0;
  const double beta = first ? 0.0 : sh.cg_beta;
  auto pk1 = [&](int q) { return first ? a.r[q] : fma(beta, a.p_old[q], a.r[q]); };
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx0 = it.c * kChunk + threadIdx.x * kVec;
    if (a.od.ell_k > 0 && idx0 + 1 < a.n) {
      // ELL: the thread's two rows' j-th entries with one 16-byte value access
      // and one 8-byte index access (consecutive lanes, consecutive rows)
      Vals<2> rr;
      rr.load(a.r + idx0);
      double c0 = rr.v[0], c1 = rr.v[1];
      if (!first) {
        Vals<2> po;
        po.load(a.p_old + idx0);
        c0 = fma(beta, po.v[0], c0);
        c1 = fma(beta, po.v[1], c1);
      }
      double q0 = 0.0, q1 = 0.0;
      for (int j = 0; j < a.od.ell_k; ++j) {
        const size_t e = (size_t)j * a.od.ell_ld + idx0;
        Vals<2> vv;
        vv.template ld<NTL>(a.od.va + e);
        const int2 cc = *reinterpret_cast<const int2 *>(a.od.ci + e);
        q0 = fma(vv.v[0], pk1(cc.x), q0);
        q1 = fma(vv.v[1], pk1(cc.y), q1);
      }
      Vals<2> pn, qv;
      pn.v[0] = c0;
      pn.v[1] = c1;
      qv.v[0] = q0;
      qv.v[1] = q1;
      pn.template st<NTS>(a.p_new + idx0);
      qv.template st<NTS>(a.q + idx0);
      acc[0] = fma(c1, q1, fma(c0, q0, acc[0]));
      continue;
    }
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= a.n) break;
      const double pc = pk1(p);
      double q = 0.0;
      if (a.od.ell_k > 0) {
        for (int j = 0; j < a.od.ell_k; ++j) {
          const size_t e = (size_t)j * a.od.ell_ld + p;
          q = fma(a.od.va[e], pk1(a.od.ci[e]), q);
        }
      } else {
        const int64_t e = a.od.rp[p + 1];
        for (int64_t j = a.od.rp[p]; j < e; ++j) q = fma(a.od.va[j], pk1(a.od.ci[j]), q);
      }
      a.p_new[p] = pc;
      a.q[p] = q;
      acc[0] = fma(pc, q, acc[0]);
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// Sweep B of iteration k.  Prologue: alpha_k = rho_k / (p_k, q) from sweep A
// (breakdown if (p_k, A p_k) <= 0).  Then x += alpha p_k, r -= alpha q and the
// product (r_{k+1}, r_{k+1}).  P: paired x updates - for even k (a.xmode kXSkip)
// x is left alone; for odd k (kXPair) x += alpha_{k-1} p_{k-1}, then alpha_k p_k,
// with p_{k-1} still in the other p buffer (the same two roundings).
// The vectors one pair of sweep B reads (x, p_k, r, q; paired updates: r, q,
// and on odd k x, p_k and p_{k-1}), loaded by cg_b_load and used by cg_b_pair.
struct CgBVals {
  Vals<2> x, p, r, q, po;
};

template <int H, bool P>
__device__ inline void cg_b_load(const CgArgs &a, int idx, bool upd, CgBVals &v) {
  constexpr bool NTL = (H & kHintLoads) != 0;
  if (!P || upd) {
    v.x.template ld<NTL>(a.x + idx);
    v.p.template ld<NTL>(a.p_new + idx);
  }
  v.r.template ld<NTL>(a.r + idx);
  v.q.template ld<NTL>(a.q + idx);
  if (P && upd) v.po.template ld<NTL>(a.p_old + idx);
}

template <int H, bool P>
__device__ inline void cg_b_pair(const CgArgs &a, int idx, double alpha, double alpha_prev,
                                 bool upd, CgBVals v, double (&acc)[1]) {
  constexpr bool NTS = (H & kHintStores) != 0;
  if constexpr (!P) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      v.x.v[k] = fma(alpha, v.p.v[k], v.x.v[k]);
      v.r.v[k] = fma(-alpha, v.q.v[k], v.r.v[k]);
      acc[0] = fma(v.r.v[k], v.r.v[k], acc[0]);
    }
    v.x.template st<NTS>(a.x + idx);
    v.r.template st<NTS>(a.r + idx);
  } else {
    if (upd) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
        v.x.v[k] = fma(alpha, v.p.v[k], fma(alpha_prev, v.po.v[k], v.x.v[k]));
      v.x.template st<NTS>(a.x + idx);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      v.r.v[k] = fma(-alpha, v.q.v[k], v.r.v[k]);
      acc[0] = fma(v.r.v[k], v.r.v[k], acc[0]);
    }
    v.r.template st<NTS>(a.r + idx);
  }
}

// Sweep B of iteration k.  Prologue: alpha_k = rho_k / (p_k, q) from sweep A
// (breakdown if (p_k, A p_k) <= 0).  Then x += alpha p_k, r -= alpha q and the
// product (r_{k+1}, r_{k+1}).  P: paired x updates - for even k (a.xmode kXSkip)
// x is left alone; for odd k (kXPair) x += alpha_{k-1} p_{k-1}, then alpha_k p_k,
// with p_{k-1} still in the other p buffer (the same two roundings).  The first
// pair's vectors are requested with the state and the partials, before the
// workgroup waits for them (not where vectors are stored non-temporally).
template <int H, bool P>
__global__ __launch_bounds__(kThreads) void cg_sweep_b_kernel(CgArgs a) {
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  WordRegs<DevState> sw;
  PartRegs<1> pr;
  words_fetch(a.st_in, sw);
  partials_fetch<1>(a.part_in, a.nparts_in, a.pstride, pr);
  const bool upd = a.xmode == kXPair;   // P: this sweep writes x
  CgBVals pre;
  bool have_pre = false;
  if constexpr ((H & kHintStores) == 0) {
    if (a.work) {
      const ChunkIter it0 = xcd_chunks(a.nchunks, a.nstream, 0, true);
      if (it0.c < it0.end) {
        const int idx = it0.at() * kChunk + threadIdx.x * kVec;
        if (idx + 1 < a.n) {
          cg_b_load<H, P>(a, idx, upd, pre);
          have_pre = true;
        }
      }
    }
  }
  words_put(sw, &sh);
  if (sh.status == kRunning) {
    partials_sum<1>(pr, a.part_in, a.nparts_in, a.pstride, lds, red);
    if (threadIdx.x == 0) {
      const double pq = red[0];
      if (!(isfinite(pq) && pq > 0.0)) {
        sh.status = kCgBreak;
        sh.last_t = a.k;
      } else {
        sh.cg_alpha_prev = sh.cg_alpha;
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
  const double alpha_prev = sh.cg_alpha_prev;
  double acc[1] = {0.0};
  // Sweep A walks the bands front to back, sweep B back to front.
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0, true); it.c < it.end; it.c += it.step) {
    const int idx = it.at() * kChunk + threadIdx.x * kVec;
    if (idx + 1 < a.n) {
      if ((H & kHintStores) == 0 && have_pre) {   // the first pair, preloaded
        have_pre = false;
        cg_b_pair<H, P>(a, idx, alpha, alpha_prev, upd, pre, acc);
        continue;
      }
      CgBVals v;
      cg_b_load<H, P>(a, idx, upd, v);
      cg_b_pair<H, P>(a, idx, alpha, alpha_prev, upd, v, acc);
    } else if (idx < a.n) {
      if (!P)
        a.x[idx] = fma(alpha, a.p_new[idx], a.x[idx]);
      else if (upd)
        a.x[idx] = fma(alpha, a.p_new[idx], fma(alpha_prev, a.p_old[idx], a.x[idx]));
      const double rv = fma(-alpha, a.q[idx], a.r[idx]);
      a.r[idx] = rv;
      acc[0] = fma(rv, rv, acc[0]);
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// ---------------------------------------------------------------------------
// Residual, segment start, scaling, operator application, copy
// ---------------------------------------------------------------------------

// (A x)_p for operator kind K: 0 the 2D stencil, 1 the 3D stencil, 2 the
// diagonal, 3 the CSR matrix of od.
template <int K>
__device__ inline double op_at(const double *x, int p, const Grid &g, const OpData &od) {
  if constexpr (K == 2) {
    return od.dg[p] * x[p];
  } else if constexpr (K == 3) {
    return CsrOp<double>{od.rp, od.ci, od.va, od.ell_k, od.ell_ld}.row(x, p);
  } else {
    return fma(K == 1 ? 6.0 : 4.0, x[p], -neighbour_sum<K == 1>(x, p, g));
  }
}

// wdiv (optional): accumulate (r_p / wdiv_p)^2 instead of r_p^2 (the
// original-space norm of a Jacobi-scaled residual, wdiv = D^{-1/2}).
template <int K>
__global__ __launch_bounds__(kThreads) void residual_kernel(const double *b, const double *x,
                                                            double *r, double *part_out, Grid g,
                                                            OpData od, const double *wdiv,
                                                            int nchunks, int nstream) {
  constexpr bool D3 = K == 1;
  __shared__ double lds[4];
  __shared__ double red[1];
  double acc[1] = {0.0};
  const ChunkOrder order = chunk_order(g, D3, kChunk);
  for (ChunkIter it = xcd_chunks(nchunks, nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx0 = order.phys(it.c) * kChunk + threadIdx.x * kVec;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= g.n) break;
      const double rv = b[p] - op_at<K>(x, p, g, od);
      if (r != nullptr) r[p] = rv;
      const double rw = wdiv != nullptr ? rv / wdiv[p] : rv;
      acc[0] = fma(rw, rw, acc[0]);
    }
  }
  store_partials<1>(acc, part_out, kMaxStream, blockIdx.x, lds, red);
}

// One workgroup: ||b - A x||^2 from the residual partials; starts a segment.
__global__ __launch_bounds__(kThreads) void start_kernel(const double *part_in, int nparts,
                                                         DevState *st, HostStatus *hs, int mode,
                                                         double tol, double rref_in,
                                                         double abs_floor) {
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
      sh.abs_tol = fmax(tol * sh.rref, abs_floor);
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
      sh.cg_alpha_prev = 0.0;
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
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
    const T v = (T)(r[p] * inv);
    if (d0) d0[p] = v;
    if (d1) d1[p] = v;
    if (d2) d2[p] = v;
  }
}

// Jacobi scaling of a solve: bs = D^{-1/2} b and y = D^{1/2} x in place (dis = D^{-1/2}).
__global__ __launch_bounds__(kThreads) void jacobi_in_kernel(const double *b, const double *dis,
                                                             double *bs, double *x, int n) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads) {
    bs[p] = b[p] * dis[p];
    x[p] = x[p] / dis[p];
  }
}

// Back to the caller's variables: x = D^{-1/2} y in place.
__global__ __launch_bounds__(kThreads) void jacobi_out_kernel(double *x, const double *dis, int n) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads)
    x[p] = x[p] * dis[p];
}

// x += d: the FP32 correction of one refinement step added to the FP64 iterate.
__global__ __launch_bounds__(kThreads) void add_correction_kernel(double *x, const float *d, int n) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < n; p += (int64_t)gridDim.x * kThreads)
    x[p] += (double)d[p];
}

// x += zeta p, one rounding to S: the x update of an odd last sweep, which the
// paired updates of the streaming sweeps leave to the end of a run.
template <typename S>
__global__ __launch_bounds__(kThreads) void x_step_kernel(S *x, const S *p, double zeta, int n) {
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kThreads)
    x[q] = (S)fma(zeta, (double)p[q], (double)x[q]);
}

template <int K>
__global__ __launch_bounds__(kThreads) void apply_kernel(const double *x, double *y, Grid g,
                                                         OpData od) {
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < g.n;
       p += (int64_t)gridDim.x * kThreads)
    y[p] = op_at<K>(x, (int)p, g, od);
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

// Launch the sweep kernel that `a` selects or, with occ not NULL, report how
// many of its workgroups a CU keeps resident (the same selection, nothing
// launched).
template <typename S, typename K>
static hipError_t launch_or_occupancy(K kernel, int grid, const SweepArgsT<S> &a, hipStream_t s,
                                      int *occ) {
  if (occ != nullptr) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, kernel, kThreads, 0);
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <int L, typename S, int H, bool P>
static hipError_t launch_sweep_lhp(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  const int grid = a.nstream + (L >= 2 ? 1 : 0);
  if (a.od.rp != nullptr)
    return launch_or_occupancy(plcg_csr_sweep_kernel<L, S, H, P>, grid, a, s, occ);
  if (a.od.dg != nullptr)
    return launch_or_occupancy(plcg_diag_sweep_kernel<L, S, H, P>, grid, a, s, occ);
  if (a.d3) return launch_or_occupancy(plcg_sweep_kernel<L, true, S, H, P>, grid, a, s, occ);
  return launch_or_occupancy(plcg_sweep_kernel<L, false, S, H, P>, grid, a, s, occ);
}

template <int L, typename S, int H>
static hipError_t launch_sweep_lh(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  switch (a.xmode) {
    case kXEvery: return launch_sweep_lhp<L, S, H, false>(a, s, occ);
    case kXSkip:
    case kXPair: return launch_sweep_lhp<L, S, H, true>(a, s, occ);
    default: return hipErrorInvalidValue;
  }
}

template <int L, typename S>
static hipError_t launch_sweep_l(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  switch (a.hint) {
    case 0: return launch_sweep_lh<L, S, 0>(a, s, occ);
    case kHintLoads: return launch_sweep_lh<L, S, kHintLoads>(a, s, occ);
    case kHintLoads | kHintStores:
      return launch_sweep_lh<L, S, kHintLoads | kHintStores>(a, s, occ);
    default: return hipErrorInvalidValue;
  }
}

template <typename S>
static hipError_t launch_sweep_any(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  if (a.od.sx != nullptr) return launch_var_sweep(a, s, occ);
  switch (a.l) {
    case 1: return launch_sweep_l<1, S>(a, s, occ);
    case 2: return launch_sweep_l<2, S>(a, s, occ);
    case 3: return launch_sweep_l<3, S>(a, s, occ);
    case 4: return launch_sweep_l<4, S>(a, s, occ);
    case 5: return launch_sweep_l<5, S>(a, s, occ);
    case 6: return launch_sweep_l<6, S>(a, s, occ);
    case 7: return launch_sweep_l<7, S>(a, s, occ);
    case 8: return launch_sweep_l<8, S>(a, s, occ);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plcg_sweep(const SweepArgsT<double> &a, hipStream_t s) {
  return launch_sweep_any<double>(a, s, nullptr);
}

hipError_t launch_plcg_sweep(const SweepArgsT<float> &a, hipStream_t s) {
  return launch_sweep_any<float>(a, s, nullptr);
}

hipError_t plcg_sweep_occupancy(const SweepArgsT<double> &a, int *per_cu) {
  return launch_sweep_any<double>(a, nullptr, per_cu);
}

hipError_t plcg_sweep_occupancy(const SweepArgsT<float> &a, int *per_cu) {
  return launch_sweep_any<float>(a, nullptr, per_cu);
}

template <int H>
static hipError_t launch_cg_a_h(const CgArgs &a, hipStream_t s) {
  if (a.od.rp != nullptr)
    hipLaunchKernelGGL((cg_csr_sweep_a_kernel<H>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  else if (a.od.dg != nullptr)
    hipLaunchKernelGGL((cg_diag_sweep_a_kernel<H>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  else if (a.d3)
    hipLaunchKernelGGL((cg_sweep_a_kernel<true, H>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((cg_sweep_a_kernel<false, H>), dim3(a.nstream), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cg_sweep_a(const CgArgs &a, hipStream_t s) {
  if (a.od.sx != nullptr) return launch_var_cg_sweep_a(a, s);
  switch (a.hint) {
    case 0: return launch_cg_a_h<0>(a, s);
    case kHintLoads: return launch_cg_a_h<kHintLoads>(a, s);
    case kHintLoads | kHintStores: return launch_cg_a_h<kHintLoads | kHintStores>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int H>
static hipError_t launch_cg_b_h(const CgArgs &a, hipStream_t s) {
  switch (a.xmode) {
    case kXEvery:
      hipLaunchKernelGGL((cg_sweep_b_kernel<H, false>), dim3(a.nstream), dim3(kThreads), 0, s, a);
      break;
    case kXSkip:
    case kXPair:
      hipLaunchKernelGGL((cg_sweep_b_kernel<H, true>), dim3(a.nstream), dim3(kThreads), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cg_sweep_b(const CgArgs &a, hipStream_t s) {
  switch (a.hint) {
    case 0: return launch_cg_b_h<0>(a, s);
    case kHintLoads: return launch_cg_b_h<kHintLoads>(a, s);
    case kHintLoads | kHintStores: return launch_cg_b_h<kHintLoads | kHintStores>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_residual(const double *b, const double *x, double *r, double *part_out, int n,
                           int nx, int ny, int nz, bool d3, const OpData &od, const double *wdiv,
                           int nchunks, int nstream, hipStream_t s) {
  if (od.sx != nullptr)
    return launch_var_residual(b, x, r, part_out, n, nx, ny, nz, d3, od, wdiv, nchunks, nstream,
                               s);
  const Grid g{n, nx, ny, nz};
  const int k = od.rp != nullptr ? 3 : od.dg != nullptr ? 2 : d3 ? 1 : 0;
  const dim3 grid(nstream), block(kThreads);
  switch (k) {
    case 3: hipLaunchKernelGGL(residual_kernel<3>, grid, block, 0, s, b, x, r, part_out, g, od, wdiv, nchunks, nstream); break;
    case 2: hipLaunchKernelGGL(residual_kernel<2>, grid, block, 0, s, b, x, r, part_out, g, od, wdiv, nchunks, nstream); break;
    case 1: hipLaunchKernelGGL(residual_kernel<1>, grid, block, 0, s, b, x, r, part_out, g, od, wdiv, nchunks, nstream); break;
    default: hipLaunchKernelGGL(residual_kernel<0>, grid, block, 0, s, b, x, r, part_out, g, od, wdiv, nchunks, nstream); break;
  }
  return hipGetLastError();
}

hipError_t launch_start(const double *part_in, int nparts, DevState *st, HostStatus *hs, int mode,
                        double tol, double rref_in, double abs_floor, hipStream_t s) {
  hipLaunchKernelGGL(start_kernel, dim3(1), dim3(kThreads), 0, s, part_in, nparts, st, hs, mode,
                     tol, rref_in, abs_floor);
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

hipError_t launch_jacobi_in(const double *b, const double *dis, double *bs, double *x, int n,
                            hipStream_t s) {
  hipLaunchKernelGGL(jacobi_in_kernel, dim3(simple_blocks(n)), dim3(kThreads), 0, s, b, dis, bs, x,
                     n);
  return hipGetLastError();
}

hipError_t launch_jacobi_out(double *x, const double *dis, int n, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_out_kernel, dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, dis, n);
  return hipGetLastError();
}

hipError_t launch_add_correction(double *x, const float *d, int n, hipStream_t s) {
  hipLaunchKernelGGL(add_correction_kernel, dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, d, n);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_x_step(S *x, const S *p, double zeta, int n, hipStream_t s) {
  hipLaunchKernelGGL(x_step_kernel<S>, dim3(simple_blocks(n)), dim3(kThreads), 0, s, x, p, zeta, n);
  return hipGetLastError();
}
template hipError_t launch_x_step<double>(double *, const double *, double, int, hipStream_t);
template hipError_t launch_x_step<float>(float *, const float *, double, int, hipStream_t);

hipError_t launch_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                        const OpData &od, hipStream_t s) {
  if (od.sx != nullptr) return launch_var_apply(x, y, n, nx, ny, nz, d3, od, s);
  const Grid g{n, nx, ny, nz};
  const int k = od.rp != nullptr ? 3 : od.dg != nullptr ? 2 : d3 ? 1 : 0;
  const dim3 grid(simple_blocks(n)), block(kThreads);
  switch (k) {
    case 3: hipLaunchKernelGGL(apply_kernel<3>, grid, block, 0, s, x, y, g, od); break;
    case 2: hipLaunchKernelGGL(apply_kernel<2>, grid, block, 0, s, x, y, g, od); break;
    case 1: hipLaunchKernelGGL(apply_kernel<1>, grid, block, 0, s, x, y, g, od); break;
    default: hipLaunchKernelGGL(apply_kernel<0>, grid, block, 0, s, x, y, g, od); break;
  }
  return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(simple_blocks((n + 1) / 2)), dim3(kThreads), 0, s, src, dst,
                     n);
  return hipGetLastError();
}

}  // namespace plcg
