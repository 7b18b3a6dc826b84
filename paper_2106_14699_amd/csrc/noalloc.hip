// cmif_compute_noalloc: cmif_compute without caller workspaces and without
// any device allocation, for callers that cannot allocate (code under graph
// capture, tight serving loops).
//
// Both workspaces (persistent tables and per-call scratch) live in one
// file-scope device array.  In host code the array's name is only a host
// stand-in, so its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// passed on; every GPU holds its own copy of the array at its own address,
// for the life of the process.  The call rebuilds its tables and clears
// its counters on every call (as cmif_compute does with a fresh scratch
// buffer), so the contents a previous call left are never read.  Calls that
// overlap in time on one GPU share the array and race: they must be ordered
// (one stream, or synchronised streams).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kernels.h"

namespace {

constexpr size_t kNoallocBytes = size_t(128) << 20;  // CMIF_NOALLOC_BYTES
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Device address of `scratch` on `dev` (the current device), looked up once.
cmif_status scratch_on(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return cmif::set_error(CMIF_ERR_NO_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return cmif::set_error(CMIF_ERR_DEVICE,
                             (std::string("hipGetSymbolAddress(scratch): ") +
                              hipGetErrorString(e)).c_str());
    }
    g_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_ptr[dev]);
  return CMIF_OK;
}

}  // namespace

extern "C" cmif_status cmif_compute_noalloc(cmif_plan_t plan,
                                            const cmif_inputs* in,
                                            const cmif_outputs* out,
                                            void* stream) {
  if (!plan || !in)
    return cmif::set_error(CMIF_ERR_INVALID_ARGUMENT, "NULL plan or inputs");
  int dev = 0;
  size_t pers = 0, scr = 0;
  uint32_t flags = 0;
  int32_t mode = 0;
  cmif_status s = cmif::plan_noalloc_info(plan, &dev, &pers, &scr, &flags, &mode);
  if (s != CMIF_OK) return s;
  if (mode == CMIF_MODE_SOFT && (flags & CMIF_FLAG_SAVE_FOR_BACKWARD))
    return cmif::set_error(CMIF_ERR_UNSUPPORTED,
                           "cmif_compute_noalloc keeps no state for "
                           "cmif_backward (SAVE_FOR_BACKWARD plans)");
  const size_t need = up256(pers) + scr;
  if (need > kNoallocBytes)
    return cmif::set_error(
        CMIF_ERR_UNSUPPORTED,
        ("the plan needs " + std::to_string(need) +
         " bytes of workspace; cmif_compute_noalloc has " +
         std::to_string(kNoallocBytes))
            .c_str());
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess)
    return cmif::set_error(CMIF_ERR_DEVICE, "hipGetDevice failed");
  if (prev != dev && hipSetDevice(dev) != hipSuccess)
    return cmif::set_error(CMIF_ERR_NO_DEVICE, "cannot select the plan's device");
  unsigned char* base = nullptr;
  s = scratch_on(dev, &base);
  if (s == CMIF_OK)
    s = cmif::compute_eager(plan, in, out, base, base + up256(pers),
                            static_cast<hipStream_t>(stream));
  if (prev != dev) (void)hipSetDevice(prev);
  return s;
}
