// sbt_create_static: a context whose device memory is a file-scope static
// device array instead of a caller-provided buffer, for callers that cannot
// allocate device memory (code under stream capture, serving loops, hosts
// that forbid hipMalloc).  The kernels are those of sbt_create; they take
// the array's device address as the base of every table and lattice.
//
// The array is kStaticBytes long and each GPU holds its own copy from the
// first call on that device until the process ends.  Its device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current; host code never passes the array's name itself (in host code it
// is a host-side stand-in, not a device address).  One context at a time
// may live in a device's array: a second call on the same device before
// sbt_destroy of the first is rejected with SBT_ERR_STATE (two live contexts
// would overwrite each other's state).  sbt_create fills everything a
// context reads before its first step (lattices, tables, counters, error
// flags), so nothing of an earlier context's contents survives.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sbt_internal.h"

namespace {

constexpr size_t kStaticBytes = SBT_STATIC_BYTES;   // 128 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
bool g_busy[kMaxDevices] = {};

}  // namespace

extern "C" {

void sbt_static_release(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev >= 0 && dev < kMaxDevices) g_busy[dev] = false;
}

sbt_status sbt_create_static(const sbt_case_desc *cases, int32_t n_cases, void *hip_stream, sbt_ctx **out) {
  if (!out) return sbt_set_error(SBT_ERR_ARG, "null output");
  *out = nullptr;
  size_t need = 0;
  sbt_status st = sbt_plan(cases, n_cases, &need);
  if (st) return st;
  if (need > kStaticBytes)
    return sbt_set_error(SBT_ERR_NOMEM, ("the cases need " + std::to_string(need) + " device bytes; the static array holds " +
                                         std::to_string(kStaticBytes)).c_str());
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return sbt_set_error(SBT_ERR_DEVICE, "no current device");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_busy[dev]) return sbt_set_error(SBT_ERR_STATE, "a context created by sbt_create_static is alive on this device");
    if (!g_ptr[dev]) {
      // this device's copy of the array (the current device is dev)
      void *p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return sbt_set_error(SBT_ERR_DEVICE, (std::string("static array address: ") + hipGetErrorString(e)).c_str());
      g_ptr[dev] = p;
    }
    base = g_ptr[dev];
    g_busy[dev] = true;
  }
  st = sbt_create_in(cases, n_cases, base, kStaticBytes, hip_stream, dev, out);
  if (st) sbt_static_release(dev);
  return st;
}

}  // extern "C"
