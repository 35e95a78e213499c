// Variable-coefficient grid operators on the single-system path (gfx950).
//
// (A u)_p = sum over the grid edges (p, q) incident to p of c_pq (u_p - u_q),
// with u = 0 outside the grid: the operator of the batched workloads, here for
// one system per solver, either Jacobi-scaled (D^{-1/2} A D^{-1/2}, unit
// diagonal and scaled edge weights: Alg. 1 with M = diag(A) in its symmetric
// form) or as given (the diagonal d_p, the sum of the edges at p, in an array of
// its own).  The kernels are those of the constant stencil with VarOp in place
// of the integer stencil: each SpMV reads two (2D) or three (3D) arrays of edge
// weights more, plus the diagonal in the unscaled form.
#include "plcg_sweep.h"

namespace plcg {

__device__ inline VarOp var_op(const OpData &od, int n, int nx, int ny, int nz, int d3) {
  return VarOp{od.sx, od.sy, od.sz, n, nx, ny, nz, d3, od.vd};
}

template <int L, typename ST, int H, bool P>
__global__ __launch_bounds__(kThreads) void plcg_var_sweep_kernel(SweepArgsT<ST> a) {
  const Grid g{a.n, a.nx, a.ny, a.nz};
  plcg_sweep<L, ST, H, P>(a, var_op(a.od, a.n, a.nx, a.ny, a.nz, a.d3),
                          a.nx % vec_of<ST>() == 0,
                          chunk_order(g, a.d3 != 0, kThreads * vec_of<ST>()));
}

// CG sweep A: p_k = r_k + beta_{k-1} p_{k-1}, formed at every unknown the
// operator reads, q = A p_k and the product (p_k, q).
template <int H>
__global__ __launch_bounds__(kThreads) void cg_var_sweep_a_kernel(CgArgs a) {
  constexpr bool NTS = (H & kHintStores) != 0;
  __shared__ double lds[4];
  __shared__ double red[1];
  __shared__ DevState sh;
  if (!cg_a_prologue(a, sh, lds, red)) return;

  const bool first = a.k == 0;
  const double beta = first ? 0.0 : sh.cg_beta;
  const VarOp op = var_op(a.od, a.n, a.nx, a.ny, a.nz, a.d3);
  const Grid g{a.n, a.nx, a.ny, a.nz};
  const ChunkOrder order = chunk_order(g, a.d3 != 0, kChunk);
  auto pk1 = [&](int q) { return first ? a.r[q] : fma(beta, a.p_old[q], a.r[q]); };
  // p_k at the pair q, q+1 (16-byte loads)
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
  const bool fast_rows = (a.nx & 1) == 0;
  const int plane = a.nx * a.ny;
  const int lane = threadIdx.x & 63;
  double acc[1] = {0.0};
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, 0); it.c < it.end; it.c += it.step) {
    const int base = order.phys(it.c) * kChunk;
    const int idx0 = base + threadIdx.x * kVec;
    if (fast_rows && base + kChunk <= a.n) {
      // A full chunk whose pairs share a row: x-neighbours from the adjacent
      // lanes, rows, planes and the y / z edge weights with 16-byte loads; each
      // unknown's terms in the order of VarOp::at.
      double c0, c1;
      pk2(idx0, c0, c1);
      const int x = idx0 % a.nx;
      const int rest = idx0 / a.nx;
      const int y = a.d3 ? rest % a.ny : rest;
      const int zz = a.d3 ? rest / a.ny : 0;
      double left = lane_prev(c1);
      double right = lane_next(c0);
      if (lane == 0 && x > 0) left = pk1(idx0 - 1);
      if (lane == 63 && x + 2 < a.nx) right = pk1(idx0 + 2);
      const int xe = rest * (a.nx + 1) + x;
      const int ye = idx0 + zz * a.nx;
      double s0 = 0.0, s1 = 0.0;
      if (x > 0) s0 = fma(op.sx[xe], left, s0);
      s0 = fma(op.sx[xe + 1], c1, s0);               // x + 1 < nx: nx is even
      s1 = fma(op.sx[xe + 1], c0, s1);
      if (x + 2 < a.nx) s1 = fma(op.sx[xe + 2], right, s1);
      double u0, u1;
      if (y > 0) {
        Vals<2> w;
        w.load(op.sy + ye);
        pk2(idx0 - a.nx, u0, u1);
        s0 = fma(w.v[0], u0, s0);
        s1 = fma(w.v[1], u1, s1);
      }
      if (y < a.ny - 1) {
        Vals<2> w;
        w.load(op.sy + ye + a.nx);
        pk2(idx0 + a.nx, u0, u1);
        s0 = fma(w.v[0], u0, s0);
        s1 = fma(w.v[1], u1, s1);
      }
      if (a.d3 && zz > 0) {
        Vals<2> w;
        w.load(op.sz + idx0);
        pk2(idx0 - plane, u0, u1);
        s0 = fma(w.v[0], u0, s0);
        s1 = fma(w.v[1], u1, s1);
      }
      if (a.d3 && zz < a.nz - 1) {
        Vals<2> w;
        w.load(op.sz + idx0 + plane);
        pk2(idx0 + plane, u0, u1);
        s0 = fma(w.v[0], u0, s0);
        s1 = fma(w.v[1], u1, s1);
      }
      Vals<2> pn, qv;
      pn.v[0] = c0;
      pn.v[1] = c1;
      if (op.dg != nullptr) {
        Vals<2> dv;
        dv.load(op.dg + idx0);
        qv.v[0] = fma(dv.v[0], c0, -s0);
        qv.v[1] = fma(dv.v[1], c1, -s1);
      } else {
        qv.v[0] = c0 - s0;
        qv.v[1] = c1 - s1;
      }
      pn.template st<NTS>(a.p_new + idx0);
      qv.template st<NTS>(a.q + idx0);
      acc[0] = fma(c1, qv.v[1], fma(c0, qv.v[0], acc[0]));
      continue;
    }
    if (idx0 + 1 < a.n) {
      Vals<2> pn, qv;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        pn.v[v] = pk1(idx0 + v);
        qv.v[v] = op.at_f(idx0 + v, pn.v[v], pk1);
        acc[0] = fma(pn.v[v], qv.v[v], acc[0]);
      }
      pn.template st<NTS>(a.p_new + idx0);
      qv.template st<NTS>(a.q + idx0);
    } else if (idx0 < a.n) {
      const double pc = pk1(idx0);
      const double q = op.at_f(idx0, pc, pk1);
      a.p_new[idx0] = pc;
      a.q[idx0] = q;
      acc[0] = fma(pc, q, acc[0]);
    }
  }
  store_partials<1>(acc, a.part_out, a.pstride, blockIdx.x, lds, red);
}

// r = b - A x (r may be NULL) and the partial sums of r.r, or of (r / wdiv)^2.
__global__ __launch_bounds__(kThreads) void var_residual_kernel(const double *b, const double *x,
                                                                double *r, double *part_out,
                                                                Grid g, OpData od, int d3,
                                                                const double *wdiv, int nchunks,
                                                                int nstream) {
  __shared__ double lds[4];
  __shared__ double red[1];
  const VarOp op = var_op(od, g.n, g.nx, g.ny, g.nz, d3);
  double acc[1] = {0.0};
  const ChunkOrder order = chunk_order(g, d3 != 0, kChunk);
  for (ChunkIter it = xcd_chunks(nchunks, nstream, 0); it.c < it.end; it.c += it.step) {
    const int idx0 = order.phys(it.c) * kChunk + threadIdx.x * kVec;
#pragma unroll
    for (int v = 0; v < kVec; ++v) {
      const int p = idx0 + v;
      if (p >= g.n) break;
      const double rv = b[p] - op.at(x, p);
      if (r != nullptr) r[p] = rv;
      const double rw = wdiv != nullptr ? rv / wdiv[p] : rv;
      acc[0] = fma(rw, rw, acc[0]);
    }
  }
  store_partials<1>(acc, part_out, kMaxStream, blockIdx.x, lds, red);
}

__global__ __launch_bounds__(kThreads) void var_apply_kernel(const double *x, double *y, Grid g,
                                                             OpData od, int d3) {
  const VarOp op = var_op(od, g.n, g.nx, g.ny, g.nz, d3);
  for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < g.n;
       p += (int64_t)gridDim.x * kThreads)
    y[p] = op.at(x, (int)p);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int L, typename S, int H>
static hipError_t var_sweep_lh(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  const int grid = a.nstream + (L >= 2 ? 1 : 0);
  switch (a.xmode) {
    case kXEvery:
      if (occ != nullptr)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, plcg_var_sweep_kernel<L, S, H, false>, kThreads, 0);
      hipLaunchKernelGGL((plcg_var_sweep_kernel<L, S, H, false>), dim3(grid), dim3(kThreads), 0, s,
                         a);
      break;
    case kXSkip:
    case kXPair:
      if (occ != nullptr)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, plcg_var_sweep_kernel<L, S, H, true>, kThreads, 0);
      hipLaunchKernelGGL((plcg_var_sweep_kernel<L, S, H, true>), dim3(grid), dim3(kThreads), 0, s,
                         a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L, typename S>
static hipError_t var_sweep_l(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  switch (a.hint) {
    case 0: return var_sweep_lh<L, S, 0>(a, s, occ);
    case kHintLoads: return var_sweep_lh<L, S, kHintLoads>(a, s, occ);
    case kHintLoads | kHintStores:
      return var_sweep_lh<L, S, kHintLoads | kHintStores>(a, s, occ);
    default: return hipErrorInvalidValue;
  }
}

template <typename S>
static hipError_t var_sweep_any(const SweepArgsT<S> &a, hipStream_t s, int *occ) {
  switch (a.l) {
    case 1: return var_sweep_l<1, S>(a, s, occ);
    case 2: return var_sweep_l<2, S>(a, s, occ);
    case 3: return var_sweep_l<3, S>(a, s, occ);
    case 4: return var_sweep_l<4, S>(a, s, occ);
    case 5: return var_sweep_l<5, S>(a, s, occ);
    case 6: return var_sweep_l<6, S>(a, s, occ);
    case 7: return var_sweep_l<7, S>(a, s, occ);
    case 8: return var_sweep_l<8, S>(a, s, occ);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_var_sweep(const SweepArgsT<double> &a, hipStream_t s, int *occ) {
  return var_sweep_any<double>(a, s, occ);
}

hipError_t launch_var_sweep(const SweepArgsT<float> &a, hipStream_t s, int *occ) {
  return var_sweep_any<float>(a, s, occ);
}

hipError_t launch_var_cg_sweep_a(const CgArgs &a, hipStream_t s) {
  switch (a.hint) {
    case 0:
      hipLaunchKernelGGL((cg_var_sweep_a_kernel<0>), dim3(a.nstream), dim3(kThreads), 0, s, a);
      break;
    case kHintLoads:
      hipLaunchKernelGGL((cg_var_sweep_a_kernel<kHintLoads>), dim3(a.nstream), dim3(kThreads), 0,
                         s, a);
      break;
    case kHintLoads | kHintStores:
      hipLaunchKernelGGL((cg_var_sweep_a_kernel<kHintLoads | kHintStores>), dim3(a.nstream),
                         dim3(kThreads), 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_var_residual(const double *b, const double *x, double *r, double *part_out,
                               int n, int nx, int ny, int nz, bool d3, const OpData &od,
                               const double *wdiv, int nchunks, int nstream, hipStream_t s) {
  hipLaunchKernelGGL(var_residual_kernel, dim3(nstream), dim3(kThreads), 0, s, b, x, r, part_out,
                     Grid{n, nx, ny, nz}, od, d3 ? 1 : 0, wdiv, nchunks, nstream);
  return hipGetLastError();
}

hipError_t launch_var_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                            const OpData &od, hipStream_t s) {
  int64_t blocks = ((int64_t)n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(var_apply_kernel, dim3((int)blocks), dim3(kThreads), 0, s, x, y,
                     Grid{n, nx, ny, nz}, od, d3 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace plcg
