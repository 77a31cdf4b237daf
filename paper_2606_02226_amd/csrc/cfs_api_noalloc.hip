// cfs_api_noalloc.hip -- cfs_chaos_game for callers that cannot allocate
// device memory (work under HIP graph capture, tight serving loops, hosts
// that forbid allocation): the binned splat's records and run tables live in
// a fixed device array of the library instead of a caller workspace, and the
// run is cut into launches whose workspace fits it.
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel (on the host that name is a
// stand-in, not a device address); the address comes from
// hipGetSymbolAddress, taken once per device on the first call with that
// device current, and is what the kernels receive.
#include <mutex>

#include "cfs.h"
#include "cfs_api_internal.hpp"

namespace cfs {
namespace {

constexpr size_t kScratchBytes = CFS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch keeps 256-byte alignment");
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the current device's).
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(CFS_E_UNSUPPORTED, "device %d is beyond the %d devices supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(scratch)");
    if (!p || reinterpret_cast<uintptr_t>(p) % 256)
      return fail(CFS_E_DEVICE, "scratch array address %p is not 256-byte aligned", p);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CFS_OK;
}

}  // namespace
}  // namespace cfs

using namespace cfs;

extern "C" int cfs_chaos_game_noalloc(const cfs_system *sys, const cfs_run *run,
                                      const cfs_image *img, void *final_points,
                                      uint8_t *last_index, uint8_t *indices, void *stream) {
  clear_error();
  ChaosCall cc;
  int rc = chaos_prepare(sys, run, img, final_points, last_index, indices, kScratchBytes, &cc);
  if (rc) return rc;
  void *ws = nullptr;
  if (cc.job.binned) {
    rc = scratch_address(&ws);
    if (rc) return rc;
    if (cc.need > kScratchBytes)  // chaos_prepare sized the launches to fit
      return fail(CFS_E_WORKSPACE, "launch needs %zu bytes of scratch, %zu available", cc.need,
                  kScratchBytes);
  }
  // no timing events: the measurement hook creates them on first use
  return chaos_launch(cc, ws, false, static_cast<hipStream_t>(stream));
}
