// Batched solves on gfx950: one launch advances every system by one step.
//
// Each system (slot) owns a fixed number of streaming workgroups, chosen from
// its size alone, plus one owner workgroup that carries the slot's scalar state
// from one launch to the next, finalises column i of G from the partial sums of
// the previous launch (Alg. 1, update of G / T / LU) and decides the slot's
// next phase.  Because the coefficients of iteration i are first used l-1
// launches later, the owner never holds up the streaming workgroups; this is
// why the batched path runs p(l)-CG with l >= 2.  A system's arithmetic does not
// depend on which other systems share the launch, so its result is bit for bit
// the same alone and in any mix.
//
// The operator is the Jacobi-scaled variable-coefficient Laplacian
// A~ = D^{-1/2} A D^{-1/2} (unit diagonal), with (A u)_p = sum_q c_pq (u_p - u_q)
// over the grid edges incident to p (u = 0 outside), stored as scaled edge
// weights; the solver works on y = D^{1/2} x.
//
// FP32-refined batches store the inner solver's vectors (bases, p and the
// correction c) in FP32 and keep y, the residual, the operator and every scalar
// in FP64: each refinement step recomputes r = D^{-1/2} b - A~ y, solves
// A~ c = r with the FP32-stored p(l)-CG to inner_tol ||r||, and adds y += c.
#include "plcg_device.h"

#include <type_traits>

namespace plcg {

__device__ inline void bstate_load(const BatchState *st, BatchState *sh) {
  WordRegs<BatchState> r;
  words_fetch(st, r);
  words_put(r, sh);
}
__device__ inline void bstate_store(const BatchState *sh, BatchState *st) {
  __syncthreads();
  const double *src = reinterpret_cast<const double *>(sh);
  double *dst = reinterpret_cast<double *>(st);
  for (int k = threadIdx.x; k < (int)(sizeof(BatchState) / 8); k += kThreads) dst[k] = src[k];
}

// Vector k of the slot's storage (elements of type T, vstride apart).
template <typename T>
__device__ inline T *svec(const SlotDesc &S, int k) {
  return reinterpret_cast<T *>(S.vec) + (size_t)k * S.vstride;
}

// Vector roles of sweep i: ring slot of z^{(l)}_j = 2l + j % R, basis k slots
// 2k and 2k+1 by index parity, p after the ring; the iterate is y (FP64) or,
// for an FP32-stored inner solve, the correction c after p.
template <int L, typename T>
__device__ inline void slot_sweep_args(const SlotDesc &S, int i, SweepArgsT<T> &a) {
  constexpr int R = L - 1 > 2 ? L - 1 : 2;
  const int t = i - L;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int j = i - k;
    a.zl[k] = j >= 0 ? svec<T>(S, 2 * L + j % R) : nullptr;
  }
  a.zl_out = svec<T>(S, 2 * L + (i + 1) % R);
#pragma unroll
  for (int k = 0; k < L; ++k) {
    a.zk_cur[k] = t >= 0 ? svec<T>(S, 2 * k + ((t + k) & 1)) : nullptr;
    a.zk_prev[k] = t >= 0 ? svec<T>(S, 2 * k + ((t + k + 1) & 1)) : nullptr;
  }
  a.copy_dst = (i < L - 1) ? svec<T>(S, 2 * (i + 1) + ((i + 1) & 1)) : nullptr;
  a.v0 = (i == L - 1) ? svec<T>(S, 0) : nullptr;
  a.p = svec<T>(S, 2 * L + R);
  a.p_out = a.p;
  a.xmode = kXEvery;
  if constexpr (std::is_same<T, double>::value)
    a.x = S.x;
  else
    a.x = svec<T>(S, 2 * L + R + 1);
  a.od = OpData{nullptr, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr};
  a.i = i;
  a.l = L;
  a.n = S.n;
}

// Owner step: carry the state, run the slot's scalar work, pick the next phase.
template <int L>
__device__ void owner_step(const BatchArgs &a, int slot, const SlotDesc &S, const BatchState *in,
                           BatchState *out, const double *part_in, BatchState *sh, double *lds,
                           double *red) {
  constexpr int ND = L + 1;
  bstate_load(in, sh);
  const int phase = sh->phase;
  if (phase == kStart || (phase == kSweep && sh->i >= 1 && sh->d.status == kRunning) ||
      phase == kFinal2)
    sum_partials<ND>(part_in, sh->nparts, kMaxStream, lds, red);
  if (threadIdx.x == 0) {
    BatchState &b = *sh;
    switch (phase) {
      case kInit:
        b.phase = kResid;
        break;
      case kResid:
        b.phase = kStart;
        break;
      case kStart: {
        // Alg. 1, first line, on the scaled system: beta = ||r~||, g_00 = 1.
        DevState &d = b.d;
        const double beta = sqrt(red[0]);
        if (b.first) {
          d.rref = beta;
          b.rref_orig = sqrt(red[1]);
          b.first = 0;
        }
        d.beta = beta;
        // FP64: Alg. 1 stops at tol ||r~_0||.  FP32-refined: the inner solve
        // stops at max(inner_tol ||r_k||, tol ||r~_0|| / 2) (the last correction
        // need not be more accurate than the outer goal); the refinement at
        // tol ||r~_0||.
        const double outer_tol = S.tol * d.rref;
        d.abs_tol = S.mixed ? fmax(S.inner_tol * beta, 0.5 * outer_tol) : outer_tol;
        d.cols = 0;
        d.last_t = -1;
        for (int c = 0; c < kGRing; ++c)
          for (int r2 = 0; r2 < kBand; ++r2) d.g[c][r2] = 0.0;
        for (int k = 0; k < kTRing; ++k) d.gam[k] = d.dlt[k] = d.eta[k] = d.zeta[k] = 0.0;
        gref(d, 0, 0) = 1.0;
        b.i = 0;
        b.m = S.maxit - b.total;
        if (!isfinite(beta)) {
          d.status = kNonFinite;
          b.reason = 4;
          b.phase = kFinal;
        } else if (beta == 0.0 || beta < outer_tol) {
          d.status = kConverged;
          b.reason = 1;
          b.phase = kFinal;
        } else if (b.reason == 3) {   // FP32-refined: restart limit hit in the last inner solve
          b.phase = kFinal;
        } else if (b.m <= 0) {
          d.status = kRunning;
          b.reason = 2;
          b.phase = kFinal;
        } else {
          d.status = kRunning;
          b.phase = kScale;
        }
        break;
      }
      case kScale:
        b.phase = kSweep;
        b.i = 0;
        break;
      case kSweep: {
        DevState &d = b.d;
        const int i = b.i;
        if (i >= 1 && d.status == kRunning) engine_column_l<L>(d, red, i, nullptr);
        // The next sweep has t' = i + 1 - l; stop once nothing is left to do.
        // FP32-refined: every end of the inner solve adds its correction
        // (kCorrect) and returns to the FP64 residual, where kStart decides.
        const int tn = i + 1 - L;
        const int done = S.mixed ? kCorrect : kFinal;
        int next = kSweep;
        if (d.status == kRunning) {
          if (tn > b.m) {
            b.total += b.m;
            b.reason = 2;
            next = done;
          }
        } else if (tn > d.last_t) {
          if (d.status == kConverged) {
            const int td = d.last_t < b.m ? d.last_t : b.m;
            b.total += td;
            b.reason = d.last_t <= b.m ? 1 : 2;
            next = done;
          } else {  // breakdown: restart from x_{t-1} (Sec. 2.2), keeping the reference norm
            b.total += d.last_t > 0 ? (d.last_t < b.m ? d.last_t : b.m) : 0;
            b.restarts += 1;
            if (b.restarts > S.max_restarts) {
              b.reason = 3;
              next = done;
            } else if (b.total >= S.maxit) {
              b.reason = 2;
              next = done;
            } else {
              next = S.mixed ? kCorrect : kResid;
            }
          }
        }
        b.phase = next;
        b.i = i + 1;
        break;
      }
      case kCorrect:
        b.outer += 1;
        b.phase = kResid;
        break;
      case kFinal:
        b.phase = kFinal2;
        break;
      case kFinal2:
        b.res_scaled = b.d.rref > 0.0 ? sqrt(red[0]) / b.d.rref : 0.0;
        b.res_orig = b.rref_orig > 0.0 ? sqrt(red[1]) / b.rref_orig : 0.0;
        b.phase = kReport;
        break;
      case kReport: {
        b.phase = kDone;
        SlotReport &rp = a.reports[slot];
        rp.reason = b.reason;
        rp.iters = b.total;
        rp.restarts = b.restarts;
        rp.res_scaled = b.res_scaled;
        rp.res_orig = b.res_orig;
        rp.rnorm0 = b.rref_orig;
        rp.outer = b.outer;
        rp.ticket = a.tickets[slot];
        rp.phase = kDone;
        break;
      }
      default:
        break;
    }
    b.nparts = S.nblocks;
  }
  bstate_store(sh, out);
}

// ST: storage type of the inner solver's vectors (double, or float for an
// FP32-refined batch).  y, b, D^{-1/2} and the edge weights are FP64 either way.
template <int L, typename ST, int H>
__global__ __launch_bounds__(kThreads) void batch_tick_kernel(BatchArgs a) {
  constexpr int ND = L + 1;
  constexpr bool kMixed = std::is_same<ST, float>::value;
  constexpr int R = L - 1 > 2 ? L - 1 : 2;
  __shared__ double lds[4 * ND];
  __shared__ double red[ND];
  __shared__ BatchState sh;
  // Odd ticks dispatch the schedule back to front, so a tick starts on the
  // systems the previous tick touched last (still in the memory-side cache).
  // A workgroup's share of the work is the same either way.
  const int2 e = a.sched[(a.tick & 1) ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
  const int slot = e.x;
  const int lb = e.y;
  const SlotDesc &S = a.slots[slot];
  const int par = a.tick & 1;
  const BatchState *in = a.state + 2 * slot + (par ^ 1);
  BatchState *out = a.state + 2 * slot + par;
  const double *part_in = a.part + (size_t)(2 * slot + (par ^ 1)) * ND * kMaxStream;
  double *part_out = a.part + (size_t)(2 * slot + par) * ND * kMaxStream;
  if (lb < 0) {
    owner_step<L>(a, slot, S, in, out, part_in, &sh, lds, red);
    return;
  }
  const int phase = in->phase;
  if (phase == kEmpty || phase == kDone || phase == kStart || phase == kReport) return;
  const VarOp op{S.sx, S.sy, S.sz, S.n, S.nx, S.ny, S.nz, S.d3, nullptr};
  double acc[ND];
#pragma unroll
  for (int m = 0; m < ND; ++m) acc[m] = 0.0;
  // one 16-byte access per thread and vector: 2 doubles or 4 floats
  constexpr int V = vec_of<ST>();
  const int step = S.nblocks * kThreads * V;
  const int start = lb * kThreads * V + threadIdx.x * V;

  if (phase == kSweep) {
    const int i = in->i;
    const int t = i - L;
    if (in->d.status != kRunning && t > in->d.last_t) return;
    Coef<L> cf;
    read_coef<L>(in->d, i, t, cf);
    SweepArgsT<ST> sa;
    slot_sweep_args<L, ST>(S, i, sa);
    using SW = Sweep<L, ST, VarOp, H>;
    // Chunk by chunk so that the FAST test is uniform over the workgroup.
    constexpr int CH = kThreads * V;
    const bool fast_rows = S.nx % V == 0;
    for (int base = lb * CH; base < S.n; base += step) {
      const int idx = base + threadIdx.x * V;
      if (fast_rows && base + CH <= S.n)
        SW::template chunk<V, true>(sa, op, idx, t, cf, acc);
      else
        SW::template chunk<V, false>(sa, op, idx, t, cf, acc);
    }
    store_partials<ND>(acc, part_out, kMaxStream, lb, lds, red);
    return;
  }
  // Setup, correction and final phases, one unknown at a time.
  ST *r0 = svec<ST>(S, 2 * L);                 // ring slot 0
  ST *v0 = svec<ST>(S, 0);                     // basis 0, slot 0
  ST *cc = kMixed ? svec<ST>(S, 2 * L + R + 1) : nullptr;   // FP32 correction
  const double inv_beta = phase == kScale ? 1.0 / in->d.beta : 0.0;
  for (int base = start; base < S.n; base += step) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = base + v;
      if (p >= S.n) break;
      if (phase == kInit) {
        S.x[p] = S.x[p] / S.dis[p];
      } else if (phase == kResid || phase == kFinal) {
        const double r = fma(S.dis[p], S.b[p], -op.at(S.x, p));
        if (!kMixed && phase == kResid) r0[p] = (ST)r;
        acc[0] = fma(r, r, acc[0]);
        const double ro = r / S.dis[p];       // D^{1/2} r~ = b - A x
        acc[1] = fma(ro, ro, acc[1]);
      } else if (phase == kScale) {
        // z_0 = r / ||r||; the FP32 path recomputes r in FP64 (the same expression as
        // kResid) instead of keeping an FP64 copy, and clears the correction.
        const double r = kMixed ? fma(S.dis[p], S.b[p], -op.at(S.x, p)) : (double)r0[p];
        const ST z = (ST)(r * inv_beta);
        r0[p] = z;
        v0[p] = z;
        if (kMixed) cc[p] = (ST)0;
      } else if (phase == kCorrect) {
        if (kMixed) S.x[p] += (double)cc[p];
      } else if (phase == kFinal2) {
        S.x[p] = S.x[p] * S.dis[p];
      }
    }
  }
  if (phase == kResid || phase == kFinal) store_partials<ND>(acc, part_out, kMaxStream, lb, lds, red);
}

template <int L, int H>
static hipError_t launch_tick_lh(const BatchArgs &a, int blocks, hipStream_t s) {
  if (a.mixed)
    hipLaunchKernelGGL((batch_tick_kernel<L, float, H>), dim3(blocks), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((batch_tick_kernel<L, double, H>), dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <int L>
static hipError_t launch_tick_l(const BatchArgs &a, int blocks, hipStream_t s) {
  switch (a.hint) {
    case 0: return launch_tick_lh<L, 0>(a, blocks, s);
    case kHintLoads | kHintStores: return launch_tick_lh<L, kHintLoads | kHintStores>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_tick(const BatchArgs &a, int blocks, hipStream_t s) {
  switch (a.l) {
    case 2: return launch_tick_l<2>(a, blocks, s);
    case 3: return launch_tick_l<3>(a, blocks, s);
    case 4: return launch_tick_l<4>(a, blocks, s);
    case 5: return launch_tick_l<5>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace plcg
