// Serving loop: continuous batching of solve requests on one batch.
//
// Requests arrive at given times (seconds from the start of the run).  The loop
// keeps a FIFO queue of arrived requests and admits from its head while the
// batch has a free slot and arena space for the request's work vectors
// (admission by HBM footprint; FIFO, so a large request at the head is not
// overtaken).  Between admissions it enqueues `ticks_per_round` launches, which
// advance every admitted solve, waits for them, and retires the solves that are
// done.  New requests join solves already in flight: continuous batching.
#include "plcg_internal.h"

#include "../../include/plcg.h"

#include <chrono>
#include <deque>
#include <map>
#include <string>
#include <thread>

using namespace plcg;

extern "C" plcg_status plcg_serve(plcg_batch *b, const int32_t *op_ids, const double *const *d_b,
                                  int32_t nops, const plcg_request *reqs, int32_t nreq,
                                  int32_t ticks_per_round, double time_limit_s, void *stream,
                                  plcg_request_outcome *out) {
  if (b == nullptr || op_ids == nullptr || d_b == nullptr || reqs == nullptr || out == nullptr ||
      nops < 1 || nreq < 0 || ticks_per_round < 1)
    return set_last_error(PLCG_E_INVALID, "bad argument");
  for (int32_t k = 0; k < nreq; ++k) {
    if (reqs[k].system < 0 || reqs[k].system >= nops)
      return set_last_error(PLCG_E_INVALID, "request names an unknown system");
    if (k > 0 && reqs[k].arrival_s < reqs[k - 1].arrival_s)
      return set_last_error(PLCG_E_INVALID, "requests must be sorted by arrival time");
    out[k] = plcg_request_outcome{};
    out[k].admit_s = -1.0;
    out[k].finish_s = -1.0;
  }
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  auto now = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
  std::deque<int32_t> queue;
  std::map<uint64_t, int32_t> inflight;   // ticket -> request
  int32_t next = 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  while (true) {
    const double t = now();
    if (t > time_limit_s) break;
    while (next < nreq && reqs[next].arrival_s <= t) queue.push_back(next++);
    while (!queue.empty()) {
      const int32_t r = queue.front();
      const plcg_request &q = reqs[r];
      uint64_t ticket = 0;
      // x0 = 0 in the caller's buffer, ordered before the launches that read it
      if (q.x != nullptr) {
        const int64_t n = batch_op_unknowns(b, op_ids[q.system]);
        if (n < 0) return set_last_error(PLCG_E_INVALID, "unknown operator");
        if (hipMemsetAsync(q.x, 0, (size_t)n * sizeof(double), st) != hipSuccess)
          return set_last_error(PLCG_E_HIP, "hipMemsetAsync(x0)");
      }
      const plcg_status s = plcg_batch_add_op(b, op_ids[q.system], d_b[q.system], q.x, q.tol,
                                              q.maxit, stream, &ticket);
      if (s == PLCG_E_BUSY) break;
      if (s != PLCG_OK) return s;
      out[r].admit_s = now();
      inflight[ticket] = r;
      queue.pop_front();
    }
    if (inflight.empty()) {
      if (next >= nreq && queue.empty()) break;
      if (queue.empty()) {
        // idle until the next arrival
        const double wait = reqs[next].arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        continue;
      }
      // a queued request does not fit even into an empty batch
      return set_last_error(PLCG_E_INVALID, "request larger than the batch arena");
    }
    plcg_status s = plcg_batch_step(b, ticks_per_round, stream);
    if (s != PLCG_OK) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return set_last_error(PLCG_E_HIP, "hipStreamSynchronize");
    for (auto it = inflight.begin(); it != inflight.end();) {
      plcg_result res;
      s = plcg_batch_poll(b, it->first, &res);
      if (s == PLCG_NOT_READY) {
        ++it;
        continue;
      }
      if (s != PLCG_OK) return s;
      out[it->second].finish_s = now();
      out[it->second].result = res;
      it = inflight.erase(it);
    }
  }
  return PLCG_OK;
}
