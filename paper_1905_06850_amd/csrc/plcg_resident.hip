// Resident kernels of libplcg: a whole run of Alg. 1 (or of classic CG) on a
// small system in ONE launch of ONE workgroup.
//
// For a few thousand unknowns an iteration moves a few hundred kilobytes, far
// less than what it costs to launch a kernel, and a device-wide reduction
// between launches is most of the iteration.  Here one workgroup of 1024
// threads keeps every vector of the method in registers (V unknowns per
// streaming thread, strided by the number of streaming threads) and shares only
// the vector the operator is applied to, through LDS.  The reductions stay inside the
// workgroup: wave_sum within each wave, then once more over the wave sums, so
// a solve is bitwise reproducible.
//
// Synchronisation per iteration (workgroup barriers):
//   p(1)-CG: 2 - the coefficients of sweep i need the products of sweep i-1;
//   p(l)-CG, l >= 2: 1 - the owner wave finalises the column of G of sweep
//            i-1's products while the other waves stream sweep i; the coefficients it
//            produces are first read l-1 iterations later (Sec. 3.1: the
//            reduction is overlapped with the next l SpMVs, here the global
//            reduction is the workgroup's);
//   CG:      3 - (p, Ap) before the x, r update, (r, r) before the next p.
// Every stop decision is taken from values all threads read after the same
// barrier, so all waves leave the loop together.
#include "plcg_device.h"

namespace plcg {

namespace {

constexpr int kResWaves = kResThreads / 64;

// Which face neighbours of unknown p exist (bits: x-1, x+1, y-1, y+1, z-1,
// z+1), found once per solve: a thread's unknowns never change.
__device__ inline int res_faces(int p, const Grid &g, bool d3) {
  const int x = p % g.nx;
  const int rest = p / g.nx;
  const int y = d3 ? rest % g.ny : rest;
  int m = (x > 0 ? 1 : 0) | (x < g.nx - 1 ? 2 : 0) | (y > 0 ? 4 : 0) | (y < g.ny - 1 ? 8 : 0);
  if (d3) {
    const int zz = rest / g.ny;
    m |= (zz > 0 ? 16 : 0) | (zz < g.nz - 1 ? 32 : 0);
  }
  return m;
}

// (A z)_p for operator kind K (0 2D stencil, 1 3D stencil, 2 diagonal, 3 CSR),
// z the LDS copy of the shared vector, zc = z_p, faces from res_faces (K <= 1),
// dp the diagonal entry (K = 2).  Same terms in the same order as the
// streaming kernels' per-unknown path (neighbour_sum, CsrOp::row).
template <int K>
__device__ inline double res_apply(const double *z, int p, double zc, const Grid &g,
                                   const OpData &od, double dp, int faces) {
  if constexpr (K <= 1) {
    double s = 0.0;
    if (faces & 1) s += z[p - 1];
    if (faces & 2) s += z[p + 1];
    if (faces & 4) s += z[p - g.nx];
    if (faces & 8) s += z[p + g.nx];
    if (K == 1) {
      if (faces & 16) s += z[p - g.nx * g.ny];
      if (faces & 32) s += z[p + g.nx * g.ny];
    }
    return fma(K == 1 ? 6.0 : 4.0, zc, -s);
  } else if constexpr (K == 2) {
    return dp * zc;
  } else {
    // CsrOp::row with 32-bit offsets (a resident matrix has fewer than 2^30
    // stored entries, padding included)
    double s = 0.0;
    if (od.ell_k > 0) {
      for (int j = 0; j < od.ell_k; ++j) {
        const int e = j * od.ell_ld + p;
        s = fma(od.va[e], z[od.ci[e]], s);
      }
    } else {
      const int e1 = (int)od.rp[p + 1];
      for (int j = (int)od.rp[p]; j < e1; ++j) s += od.va[j] * z[od.ci[j]];
    }
    return s;
  }
}

// Sum of the wave sums of product m: lane w loads wave w's sum and the wave
// adds them with wave_sum, so every lane of every wave that calls this gets the
// same bits.
template <int ND>
__device__ inline double waves_total(const double (*red)[ND], int m, int nwaves = kResWaves) {
  const int lane = threadIdx.x & 63;
  return wave_sum(lane < nwaves ? red[lane][m] : 0.0);
}

__device__ inline void res_state_load(const DevState *src, DevState *dst) {
  const double *s = reinterpret_cast<const double *>(src);
  double *d = reinterpret_cast<double *>(dst);
  for (int k = threadIdx.x; k < (int)(sizeof(DevState) / 8); k += kResThreads) d[k] = s[k];
}

__device__ inline void res_state_store(const DevState *src, DevState *dst) {
  const double *s = reinterpret_cast<const double *>(src);
  double *d = reinterpret_cast<double *>(dst);
  for (int k = threadIdx.x; k < (int)(sizeof(DevState) / 8); k += kResThreads) d[k] = s[k];
}

}  // namespace

// One run of Alg. 1: sweeps i = 0 .. imax, with the same per-unknown arithmetic
// as Sweep<L>::steady / startup (K1, K4, K6, K5) and the same scalar engine
// (engine_column_l: update of G, Eqs. haa1/haa3, LU, breakdown and stopping
// tests).
//
// Wave 0 is the owner: it adds up the products of each sweep and finalises
// the column of G (thread 0), holding no vector data.  Waves 1..15 stream:
// thread s = threadIdx.x - 64 holds unknowns s, s + 960, ... (V of them), with
// z^{(l)} as a register ring of R slots (slot h = z^{(l)}_{i-h}) and basis
// k < l as two registers (z^{(k)}_{t+k}, z^{(k)}_{t+k-1}).  The two roles run
// separate loops with the same barriers and the same stop decision, so the
// registers of the engine and of the vectors are never live together.
template <int L, int V, int K>
__global__ __launch_bounds__(kResThreads) void plcg_resident_kernel(ResArgs a) {
  constexpr int ND = L + 1;
  constexpr int R = L - 1 > 2 ? L - 1 : 2;
  constexpr int NS = kResThreads - 64;         // streaming threads
  __shared__ double zs[2][kResMax];            // z^{(l)}_i by sweep parity
  __shared__ double red[2][kResWaves][ND];     // wave sums by sweep parity (waves 1..15)
  __shared__ DevState sh;                      // scalar state, written by thread 0 only
  __shared__ int ctl[2][2];                    // (status, last_t) after column i, by parity
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = a.n;

  res_state_load(a.st_in, &sh);
  __syncthreads();
  // Sweep i stops (all waves, same values after the same barrier) once the
  // solve has stopped and x_{last_t} is formed: sweeps past the stop change
  // nothing.  L = 1 decides on the state after column i, L >= 2 on the state
  // after column i-1, as the streaming kernels do.
  auto stop = [&](int i) {
    const int q = L == 1 ? (i & 1) : ((i - 1) & 1);
    return ctl[q][0] != kRunning && i - L > ctl[q][1];
  };

  if (wave == 0) {
    if (tid == 0) {
      ctl[1][0] = sh.status;
      ctl[1][1] = sh.last_t;
    }
    __syncthreads();
    // l = 1: thread 0 reads the state entries of column i+1 while the other
    // waves run sweep i (engine_gather_1), so that after the products arrive
    // the column step is arithmetic only.
    EngineIn1 in1{};
    for (int i = 0; i <= a.imax; ++i) {
      // column i of G from the products of sweep i-1
      if (i >= 1 && sh.status == kRunning) {
        double raw[ND];
#pragma unroll
        for (int m = 0; m < ND; ++m) raw[m] = waves_total<ND>(red[(i - 1) & 1], m, kResWaves - 1);
        if (tid == 0) {
          if constexpr (L == 1)
            engine_column_1(sh, in1, raw, i, a.hist);
          else
            engine_column_l<L>(sh, raw, i, a.hist);
        }
      }
      if (tid == 0) {
        ctl[i & 1][0] = sh.status;
        ctl[i & 1][1] = sh.last_t;
      }
      if (L == 1) __syncthreads();   // sweep i needs column i at once
      if (stop(i)) break;
      if constexpr (L == 1) {
        if (tid == 0) {
          in1 = engine_gather_1(sh, i + 1);
          asm volatile("" ::"v"(in1.g_tt), "v"(in1.g_pt), "v"(in1.dlt1), "v"(in1.gam1),
                       "v"(in1.eta1), "v"(in1.zeta1), "v"(in1.sigma0), "v"(in1.beta),
                       "v"(in1.abs_tol), "v"(in1.hist_cap));
        }
      }
      __syncthreads();
    }
  } else {
    const int sidx = tid - 64;
    const Grid g{n, a.nx, a.ny, a.nz};
    double zl[R][V], zk[L][2][V], pv[V], xv[V], dd[V];
    int fc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = v * NS + sidx;
      const bool in = p < n;
      const double z0 = in ? a.z0[p] : 0.0;
      fc[v] = (K <= 1 && in) ? res_faces(p, g, K == 1) : 0;
#pragma unroll
      for (int h = 0; h < R; ++h) zl[h][v] = h == 0 ? z0 : 0.0;
#pragma unroll
      for (int k = 0; k < L; ++k) {
        zk[k][0][v] = k == 0 ? z0 : 0.0;   // z^{(0)}_0 = u_0 / ||u_0||
        zk[k][1][v] = 0.0;
      }
      pv[v] = 0.0;
      xv[v] = in ? a.x[p] : 0.0;
      dd[v] = (K == 2 && in) ? a.od.dg[p] : 0.0;
      if (in) zs[0][p] = z0;
    }
    __syncthreads();
    for (int i = 0; i <= a.imax; ++i) {
      const int t = i - L;
      if (L == 1) __syncthreads();
      if (stop(i)) break;
      Coef<L> cf;
      read_coef<L>(sh, i, t, cf);
      const double *zcur = zs[i & 1];
      double *znext = zs[(i + 1) & 1];
      double acc[ND];
#pragma unroll
      for (int m = 0; m < ND; ++m) acc[m] = 0.0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int p = v * NS + sidx;
        if (p < n) {
          const double zc = zl[0][v];
          const double w = res_apply<K>(zcur, p, zc, g, a.od, dd[v], fc[v]);
          double zn;
          if (t >= 0) {
            // z_{i+1} = (A z_i - gamma_t z_i - delta_{t-1} z_{i-1}) / delta_t
            const double zp = zl[1][v];
            zn = fma(-cf.dm1, zp, fma(-cf.gam, zc, w)) * cf.inv_del;
#pragma unroll
            for (int m = 1; m <= L - 3; ++m) acc[m] = fma(zn, zl[L - 1 - m][v], acc[m]);
            // bases k = l-1 .. 0, each from the values before this sweep
            double above = zc, vt = 0.0, vnew = 0.0;
#pragma unroll
            for (int k = L - 1; k >= 0; --k) {
              const double ck = zk[k][0][v];
              const double pk = t >= 1 ? zk[k][1][v] : 0.0;
              const double sk = cf.sig[k] - cf.gam;
              const double nk = fma(-cf.dm1, pk, fma(sk, ck, above)) * cf.inv_del;
              zk[k][1][v] = ck;
              zk[k][0][v] = nk;
              above = ck;
              if (k == 0) {
                vt = ck;
                vnew = nk;
              }
            }
            // x_t = x_{t-1} + zeta_{t-1} p_{t-1}, p_t = (v_t - delta_{t-1} p_{t-1}) / eta_t
            if (t == 0) {
              pv[v] = vt * cf.inv_eta;
            } else {
              xv[v] = fma(cf.zm1, pv[v], xv[v]);
              pv[v] = fma(-cf.dm1, pv[v], vt) * cf.inv_eta;
            }
            acc[0] = fma(zn, vnew, acc[0]);
            acc[L] = fma(zn, zn, acc[L]);
            if (L >= 2) acc[L - 1] = fma(zn, zc, acc[L - 1]);
            if (L >= 3) acc[L - 2] = fma(zn, zp, acc[L - 2]);
          } else {
            // start-up: z_{i+1} = (A - sigma_i) z_i, copied into basis i+1
            zn = fma(-cf.sigma_i, zc, w);
#pragma unroll
            for (int m = 1; m <= L - 2; ++m) {
              const int h = L - 1 - m;
              if (h <= i) acc[m] = fma(zn, zl[h][v], acc[m]);
            }
            if (i == L - 1) acc[0] = fma(zn, zk[0][0][v], acc[0]);
#pragma unroll
            for (int k = 1; k < L; ++k)
              if (i == k - 1) zk[k][0][v] = zn;
            acc[L] = fma(zn, zn, acc[L]);
            if (L >= 2) acc[L - 1] = fma(zn, zc, acc[L - 1]);
          }
#pragma unroll
          for (int h = R - 1; h >= 1; --h) zl[h][v] = zl[h - 1][v];
          zl[0][v] = zn;
          znext[p] = zn;
        }
      }
      // the l+1 products of sweep i, one sum per streaming wave
#pragma unroll
      for (int m = 0; m < ND; ++m) {
        const double s = wave_sum(acc[m]);
        if (lane == 0) red[i & 1][wave - 1][m] = s;
      }
      __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = v * NS + sidx;
      if (p < n) a.x[p] = xv[v];
    }
  }
  __syncthreads();
  res_state_store(&sh, a.st_out);
  if (tid == 0) publish(sh, a.hs, sh.cols >= 1 ? fabs(sh.zeta[(sh.cols - 1) % kTRing]) : sh.beta,
                        sh.cols);
}

// Classic CG (Sec. 2.1) on a resident system: iterations k = 0 .. imax - 1 and
// the stopping test of iterate imax, with the arithmetic of the streaming
// sweeps A and B: p_k = r_k + beta_{k-1} p_{k-1}, q = A p_k, alpha = rho_k /
// (p_k, q), x += alpha p_k, r -= alpha q, rho_{k+1} = (r, r).  Every thread
// forms the scalars itself from the same wave sums.
template <int V, int K>
__global__ __launch_bounds__(kResThreads) void cg_resident_kernel(ResArgs a) {
  __shared__ double ps[kResMax];
  __shared__ double red_pq[kResWaves][1];
  __shared__ double red_rr[kResWaves][1];
  __shared__ DevState sh;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int n = a.n;
  const Grid g{n, a.nx, a.ny, a.nz};

  res_state_load(a.st_in, &sh);
  double rv[V], pv[V], xv[V], qv[V], dd[V];
  int fc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int p = v * kResThreads + tid;
    const bool in = p < n;
    fc[v] = (K <= 1 && in) ? res_faces(p, g, K == 1) : 0;
    rv[v] = in ? a.z0[p] : 0.0;   // r_0 = b - A x_0
    xv[v] = in ? a.x[p] : 0.0;
    dd[v] = (K == 2 && in) ? a.od.dg[p] : 0.0;
    pv[v] = 0.0;
    qv[v] = 0.0;
  }
  __syncthreads();
  double rho = sh.cg_rho, beta = 0.0;
  const double abs_tol = sh.abs_tol;
  int status = sh.status, last_t = sh.last_t, cols = sh.cols;

  for (int k = 0; status == kRunning; ++k) {
    if (k >= 1) {
      const double rr = waves_total<1>(red_rr, 0);
      cols = k;
      last_t = k;
      if (!isfinite(rr)) {
        status = kCgBreak;
        break;
      }
      beta = rr / rho;
      rho = rr;
      if (sqrt(rho) < abs_tol) {
        status = kConverged;
        break;
      }
    }
    if (k >= a.imax) break;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = v * kResThreads + tid;
      if (p < n) {
        pv[v] = k == 0 ? rv[v] : fma(beta, pv[v], rv[v]);
        ps[p] = pv[v];
      }
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = v * kResThreads + tid;
      if (p < n) {
        qv[v] = res_apply<K>(ps, p, pv[v], g, a.od, dd[v], fc[v]);
        acc = fma(pv[v], qv[v], acc);
      }
    }
    {
      const double s = wave_sum(acc);
      if (lane == 0) red_pq[wave][0] = s;
    }
    __syncthreads();
    const double pq = waves_total<1>(red_pq, 0);
    if (!(isfinite(pq) && pq > 0.0)) {
      status = kCgBreak;
      last_t = k;
      break;
    }
    const double alpha = rho / pq;
    acc = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int p = v * kResThreads + tid;
      if (p < n) {
        xv[v] = fma(alpha, pv[v], xv[v]);
        rv[v] = fma(-alpha, qv[v], rv[v]);
        acc = fma(rv[v], rv[v], acc);
      }
    }
    {
      const double s = wave_sum(acc);
      if (lane == 0) red_rr[wave][0] = s;
    }
    __syncthreads();
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int p = v * kResThreads + tid;
    if (p < n) a.x[p] = xv[v];
  }
  if (tid == 0) {
    sh.status = status;
    sh.last_t = last_t;
    sh.cols = cols;
    sh.cg_rho = rho;
    sh.cg_beta = beta;
  }
  __syncthreads();
  res_state_store(&sh, a.st_out);
  if (tid == 0) publish(sh, a.hs, sqrt(rho), 2 * cols);
}

namespace {

template <int L, int K, int V>
hipError_t launch_plcg_resident_lkv(const ResArgs &a, hipStream_t s) {
  if constexpr (V <= res_vmax(L, K)) {
    hipLaunchKernelGGL((plcg_resident_kernel<L, V, K>), dim3(1), dim3(kResThreads), 0, s, a);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int L, int K>
hipError_t launch_plcg_resident_lk(const ResArgs &a, int v, hipStream_t s) {
  switch (v) {
    case 1: return launch_plcg_resident_lkv<L, K, 1>(a, s);
    case 2: return launch_plcg_resident_lkv<L, K, 2>(a, s);
    case 3: return launch_plcg_resident_lkv<L, K, 3>(a, s);
    case 4: return launch_plcg_resident_lkv<L, K, 4>(a, s);
    case 5: return launch_plcg_resident_lkv<L, K, 5>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L>
hipError_t launch_plcg_resident_l(const ResArgs &a, int v, int kind, hipStream_t s) {
  switch (kind) {
    case 0: return launch_plcg_resident_lk<L, 0>(a, v, s);
    case 1: return launch_plcg_resident_lk<L, 1>(a, v, s);
    case 2: return launch_plcg_resident_lk<L, 2>(a, v, s);
    case 3: return launch_plcg_resident_lk<L, 3>(a, v, s);
    default: return hipErrorInvalidValue;
  }
}

template <int V>
hipError_t launch_cg_resident_v(const ResArgs &a, int kind, hipStream_t s) {
  const dim3 grid(1), block(kResThreads);
  switch (kind) {
    case 0: hipLaunchKernelGGL((cg_resident_kernel<V, 0>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((cg_resident_kernel<V, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((cg_resident_kernel<V, 2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((cg_resident_kernel<V, 3>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int resident_width(int method_plcg, int l, int kind, int n) {
  if (n < 1 || n > kResMax || kind < 0 || kind > 3) return 0;
  const int per = method_plcg ? kResThreads - 64 : kResThreads;
  const int v = (n + per - 1) / per;
  if (method_plcg && (l < 1 || l > kLMax || v > res_vmax(l, kind))) return 0;
  return v <= 5 ? v : 0;
}

hipError_t launch_plcg_resident(const ResArgs &a, int l, int kind, hipStream_t s) {
  const int v = resident_width(1, l, kind, a.n);
  switch (l) {
    case 1: return launch_plcg_resident_l<1>(a, v, kind, s);
    case 2: return launch_plcg_resident_l<2>(a, v, kind, s);
    case 3: return launch_plcg_resident_l<3>(a, v, kind, s);
    case 4: return launch_plcg_resident_l<4>(a, v, kind, s);
    case 5: return launch_plcg_resident_l<5>(a, v, kind, s);
    case 6: return launch_plcg_resident_l<6>(a, v, kind, s);
    case 7: return launch_plcg_resident_l<7>(a, v, kind, s);
    case 8: return launch_plcg_resident_l<8>(a, v, kind, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cg_resident(const ResArgs &a, int kind, hipStream_t s) {
  switch (resident_width(0, 1, kind, a.n)) {
    case 1: return launch_cg_resident_v<1>(a, kind, s);
    case 2: return launch_cg_resident_v<2>(a, kind, s);
    case 3: return launch_cg_resident_v<3>(a, kind, s);
    case 4: return launch_cg_resident_v<4>(a, kind, s);
    case 5: return launch_cg_resident_v<5>(a, kind, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace plcg
