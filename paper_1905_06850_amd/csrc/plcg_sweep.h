// Kernel bodies shared by the translation units of the single-system path:
// the p(l)-CG sweep over any operator and the prologue of CG's sweep A.
#pragma once

#include "plcg_device.h"

namespace plcg {

// Body of the p(l)-CG sweep for every operator.  Each thread takes V =
// 16 / sizeof(ST) consecutive unknowns of a chunk (one 16-byte access per
// vector: 2 doubles, or 4 floats for the FP32-stored inner solver).
// fast_rows: full chunks may take the operator's FAST form; order: the chunk
// visiting order.
template <int L, typename ST, int H, bool P, typename Op>
__device__ inline void plcg_sweep(const SweepArgsT<ST> &a, const Op &op, bool fast_rows,
                                  const ChunkOrder &order) {
  constexpr int V = vec_of<ST>();
  constexpr int CH = kThreads * V;
  using S = Sweep<L, ST, Op, H, P>;
  constexpr int ND = S::ND;
  __shared__ double lds[4 * ND];
  __shared__ double red[ND];
  __shared__ DevState sh;

  // Workgroup 0 owns the scalar state and carries it from launch i-1 to launch
  // i.  For l = 1 every workgroup finalises column i itself (this launch needs
  // it); for l >= 2 only workgroup 0 does, and it streams nothing.
  const bool owner = blockIdx.x == 0;
  const int i = a.i;
  const int t = i - L;
  // The state and the previous sweep's partials, requested together (the
  // partials before the status says whether they are needed), then column i.
  // Sweeps with cache hints may run up to kSweepStream workgroups; up to three
  // products their partials are all requested at once, beyond that (l >= 3,
  // where only the owner sums) those past kMaxStream one at a time, in the same
  // order, so that the owner's registers do not raise the kernel's count.
  constexpr int PER = H != 0 && ND <= 3 ? kSweepPer : kPartPer;
  WordRegs<DevState> sw;
  PartRegs<ND, PER> pr;
  auto engine_fetch = [&]() {
    words_fetch(a.st_in, sw);
    partials_fetch<ND, PER>(a.part_in, a.nparts_in, a.pstride, pr);
  };
  auto engine_step = [&]() {
    words_put(sw, &sh);
    if (i >= 1 && a.nparts_in > 0 && sh.status == kRunning) {
      if constexpr (L == 1) {
        // The state entries of the column step are read from LDS before the
        // partial sums, taken as used right away, so their reads are done
        // while the sums run; thread 0 then only computes.
        const EngineIn1 in = engine_gather_1(sh, i);
        asm volatile("" ::"v"(in.g_tt), "v"(in.g_pt), "v"(in.dlt1), "v"(in.gam1), "v"(in.eta1),
                     "v"(in.zeta1), "v"(in.sigma0), "v"(in.beta), "v"(in.abs_tol),
                     "v"(in.hist_cap));
        partials_sum<ND, PER>(pr, a.part_in, a.nparts_in, a.pstride, lds, red);
        if (threadIdx.x == 0) engine_column_1(sh, in, red, i, owner ? a.hist : nullptr);
      } else {
        partials_sum<ND, PER>(pr, a.part_in, a.nparts_in, a.pstride, lds, red);
        if (threadIdx.x == 0) engine_column_l<L>(sh, red, i, owner ? a.hist : nullptr);
      }
      __syncthreads();
    }
    if (owner) {
      state_store(&sh, a.st_out);
      if (threadIdx.x == 0) publish(sh, a.hs, fabs(sh.zeta[(i + kTRing - 1) % kTRing]), i);
    }
  };
  if constexpr (L >= 2) {
    if (owner) {
      engine_fetch();
      engine_step();
      return;
    }
  } else {
    engine_fetch();
  }
  // The streaming workgroups then request their first chunk's vectors and the
  // operator's data beyond them (Op::Halo: the wave-edge neighbours and rows of
  // a 2D stencil, a diagonal's entries) before the scalar state is read (it
  // decides only whether the sweep streams and with which coefficients), so
  // the round trips overlap: vector loads complete in order, and a workgroup
  // barrier does not wait for them (for l = 1 they follow the state and partial
  // loads, which are waited for first).  The chunk is computed from those
  // registers with the same arithmetic.  Not for sweeps
  // that store non-temporally (vectors of 96 MiB and more, where it was
  // measured slower), and not for FP32 storage, whose four values per thread
  // and vector, held as doubles, would double the sweep's registers (the 3D
  // p(3) sweep: 91 -> 171 VGPRs, two waves per SIMD instead of four).
  constexpr bool kPreload = L <= 3 && (H & kHintStores) == 0 && sizeof(ST) == 8;
  typename S::template Loads<V> pre;
  bool have_pre = false;
  if constexpr (kPreload) {
    if (t >= 0 && a.work) {
      const ChunkIter it0 = xcd_chunks(a.nchunks, a.nstream, L == 1 ? 0 : 1, (i & 1) != 0);
      if (it0.c < it0.end) {
        const int base = order.phys(it0.at()) * CH;
        if (fast_rows && base + CH <= a.n) {
          S::template steady_load<V>(a, op, base + threadIdx.x * V, t, pre);
          have_pre = true;
        }
      }
    }
  }
  if constexpr (L == 1) engine_step();
  if (!a.work) return;

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
    // The coefficients are taken as used here, before the status test: kept
    // after it, their loads were issued only once the status had arrived (a
    // second round trip).
    asm volatile("" ::"v"(cf.gam), "v"(cf.dm1), "v"(cf.inv_del), "v"(cf.inv_eta), "v"(cf.zm1),
                 "v"(cf.zm2), "v"(cf.sigma_i));
#pragma unroll
    for (int k = 0; k < L; ++k) asm volatile("" ::"v"(cf.sig[k]));
  }
  // Sweeps past the stop change nothing (the solve's x is x_{last_t}).
  if (status != kRunning && t > last_t) return;

  double acc[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) acc[m] = 0.0;
  const int first = L == 1 ? 0 : 1;
  for (ChunkIter it = xcd_chunks(a.nchunks, a.nstream, first, (i & 1) != 0); it.c < it.end;
       it.c += it.step) {
    const int base = order.phys(it.at()) * CH;
    const int idx = base + threadIdx.x * V;
    if constexpr (kPreload) {
      if (have_pre) {   // the first chunk, preloaded (a full chunk on the fast path)
        have_pre = false;
        S::template steady<V, true, true>(a, op, idx, t, cf, acc, &pre);
        continue;
      }
    }
    if (fast_rows && base + CH <= a.n)
      S::template chunk<V, true>(a, op, idx, t, cf, acc);
    else
      S::template chunk<V, false>(a, op, idx, t, cf, acc);
  }
  store_partials<ND>(acc, a.part_out, a.pstride, blockIdx.x - first, lds, red);
}

// Sweep A of iteration k.  Prologue (every workgroup): rho_k = (r_k, r_k) from
// sweep B of iteration k-1, beta_{k-1} = rho_k / rho_{k-1}, stopping test
// ||r_k|| < tol ||r_0||.  Then p_k = r_k + beta_{k-1} p_{k-1} (p_0 = r_0),
// q = A p_k and the product (p_k, q).
//
// The prologue in two parts, so that a sweep can request its first chunk's
// vectors in between: cg_a_fetch requests the state and sweep B's partials
// (before the status says whether they are needed), cg_a_finish waits for them
// and returns false when nothing is streamed.
struct CgPrologue {
  WordRegs<DevState> sw;
  PartRegs<1> pr;
};

__device__ inline void cg_a_fetch(const CgArgs &a, CgPrologue &f) {
  words_fetch(a.st_in, f.sw);
  partials_fetch<1, kPartPer>(a.part_in, a.nparts_in, a.pstride, f.pr);
}

__device__ inline bool cg_a_finish(const CgArgs &a, CgPrologue &f, DevState &sh, double *lds,
                                   double *red) {
  words_put(f.sw, &sh);
  if (a.k >= 1 && sh.status == kRunning) {
    partials_sum<1, kPartPer>(f.pr, a.part_in, a.nparts_in, a.pstride, lds, red);
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
  return sh.status == kRunning && a.work;
}

__device__ inline bool cg_a_prologue(const CgArgs &a, DevState &sh, double *lds, double *red) {
  CgPrologue f;
  cg_a_fetch(a, f);
  return cg_a_finish(a, f, sh, lds, red);
}

}  // namespace plcg
