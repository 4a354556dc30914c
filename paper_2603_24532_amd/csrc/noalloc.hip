// mbpt_integrate_noalloc: integration with the device state held in a static
// device array instead of a caller-bound workspace, for callers that cannot
// allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mbpt_vegas.h"
#include "runtime.hpp"

// Every GPU the library runs on holds one copy of this array until the
// process ends.  Host code never passes its name to a kernel or a copy: the
// name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[MBPT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

extern "C" int mbpt_integrate_noalloc(mbpt_task_set *set, uint64_t samples_per_iter, int iters,
                                      mbpt_result *per_task, mbpt_result *total) {
  if (!set || iters < 1 || samples_per_iter < 2) return MBPT_EINVAL;
  mbpt_context *ctx = set->ctx;
  const int dev = ctx->desc.device;
  if (dev < 0 || dev >= kMaxDevices) return MBPT_EINVAL;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return mbpt::hip_fail(ctx, e, "hipGetDevice");
  if (prev != dev) {
    e = hipSetDevice(dev);
    if (e != hipSuccess) return mbpt::hip_fail(ctx, e, "hipSetDevice");
  }
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        if (prev != dev) (void)hipSetDevice(prev);
        return mbpt::hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                              "hipGetSymbolAddress(scratch)");
      }
      g_scratch[dev] = p;
    }
    base = g_scratch[dev];
  }
  const int rc = mbpt::integrate_in(set, base, MBPT_NOALLOC_SCRATCH_BYTES, samples_per_iter,
                                    iters, per_task, total);
  if (prev != dev) (void)hipSetDevice(prev);
  return rc;
}
