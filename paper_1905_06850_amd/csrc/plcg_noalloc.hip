// plcg_solve_noalloc: a solve that allocates nothing, for callers that cannot
// call hipMalloc (tight serving loops, harnesses that forbid allocation).
//
// Its workspace - the work vectors of the method, the partial sums of the
// multi-dot reductions, the two copies of the scalar state and the progress
// record - is carved from `scratch`, a file-scope device array of
// PLCG_NOALLOC_BYTES.  Every GPU the library runs on holds its own copy of the
// array (at its own address) until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current and
// kept in g_scratch[device].  Calls on one device share the array and leave
// their contents in it; each call starts its scalar state afresh and clears
// what must start at zero.  Calls on one device are serialised here (a second
// thread waits until the first call has returned), so they never overlap
// within the process.
#include "plcg_internal.h"

#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchBytes = (size_t)PLCG_NOALLOC_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu[kMaxDevices];
void *g_scratch[kMaxDevices] = {};

}  // namespace

extern "C" {

plcg_status plcg_solve_noalloc(const plcg_operator_desc *op, const plcg_config *cfg,
                               const double *d_b, double *d_x, double tol, int32_t maxit,
                               void *stream, plcg_result *out) {
  // Argument and size checks first: they need no device.
  plcg_status e = plcg::check_workspace_solve(op, cfg, kScratchBytes);
  if (e != PLCG_OK) return e;
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess)
    return plcg::set_last_error(PLCG_E_HIP,
                                (std::string("hipGetDevice: ") + hipGetErrorString(he)).c_str());
  if (dev < 0 || dev >= kMaxDevices)
    return plcg::set_last_error(PLCG_E_INVALID, "device index beyond the supported 64");
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  if (g_scratch[dev] == nullptr) {
    void *ptr = nullptr;
    he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (he != hipSuccess || ptr == nullptr)
      return plcg::set_last_error(
          PLCG_E_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(he))
                          .c_str());
    g_scratch[dev] = ptr;
  }
  return plcg::solve_in_workspace(op, cfg, g_scratch[dev], kScratchBytes, d_b, d_x, tol, maxit,
                                  stream, out);
}

}  // extern "C"
