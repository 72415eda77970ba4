// Allocation-free filtered backprojection: lamino_fbp with the plan's tables
// and workspace placed in a file-scope device array instead of caller
// buffers, for callers that cannot allocate device memory.
//
// The array is one per device (each GPU the library runs on holds its own
// copy until the process ends).  Host code never passes the array's name to
// a kernel or a copy: its per-device address comes from hipGetSymbolAddress
// once per device, with that device current, and only that address is used.
// Every call on a device shares the array, which keeps the last call's
// contents: calls that overlap on one device race.  Nothing in it has to
// start at zero (every intermediate of the backprojection is written in full
// before it is read).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <string>

#include "lamino_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[LAMINO_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Address of this device's copy of `scratch` (looked up once per device).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int lamino_fbp_noalloc(const lamino_plan_t* p, const void* d_data, float* d_vol,
                                  void* stream) {
  if (!p) return lam::api_fail(LAMINO_E_INVALID, "lamino_fbp_noalloc: NULL plan");
  if (!d_data || !d_vol)
    return lam::api_fail(LAMINO_E_INVALID, "lamino_fbp_noalloc: NULL data or volume pointer");
  if (p->spill_D || p->spill_g)
    return lam::api_fail(LAMINO_E_UNSUPPORTED,
                         "lamino_fbp_noalloc: the plan keeps intermediates in host memory");
  const size_t tables = align256(p->table_bytes);
  const size_t need = tables + p->work_bytes;
  if (need > (size_t)LAMINO_SCRATCH_BYTES)
    return lam::api_fail(LAMINO_E_BUDGET,
                         "lamino_fbp_noalloc: the plan needs %zu bytes of device scratch, above "
                         "the limit of %zu (plan with opts.hbm_budget <= %zu)",
                         need, (size_t)LAMINO_SCRATCH_BYTES, (size_t)LAMINO_SCRATCH_BYTES - tables);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lam::api_fail(LAMINO_E_HIP, "lamino_fbp_noalloc: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return lam::api_fail(LAMINO_E_UNSUPPORTED, "lamino_fbp_noalloc: device %d", dev);
  void* base = nullptr;
  e = scratch_address(dev, &base);
  if (e != hipSuccess)
    return lam::api_fail(LAMINO_E_HIP, "lamino_fbp_noalloc: hipGetSymbolAddress: %s",
                         hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the plan's table image goes to the front of the array on the call stream
  e = hipMemcpyAsync(base, p->host_tables.data(), p->table_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return lam::api_fail(LAMINO_E_HIP, "lamino_fbp_noalloc: table upload: %s", hipGetErrorString(e));
  lam::BackprojOpts o;
  o.tables = base;
  o.work = static_cast<char*>(base) + tables;
  o.timing = false;
  e = lam::run_backprojection(p, d_data, d_vol, true, s, o);
  if (e != hipSuccess)
    return lam::api_fail(LAMINO_E_HIP, "lamino_fbp_noalloc: %s", hipGetErrorString(e));
  return LAMINO_OK;
}
