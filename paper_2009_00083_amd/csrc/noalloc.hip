// Fixed device scratch of the allocation-free entry point
// (pcrit_classify_noalloc): a file-scope device array, one copy per GPU,
// held until the process ends.
//
// Host code never passes the array's name to a kernel or a copy: in host
// code the name stands for a host-side shadow, not a device address.  The
// device address of each GPU's copy is looked up once, with that device
// current, by noalloc_scratch_init (called from pcrit_create), and every
// later use goes through the stored pointer.
#include <mutex>

#include "pcrit_internal.h"

namespace pcrit {
namespace {

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the scratch array (the caller has made
// `device` current).  Returns hipSuccess once the address is known.
hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace pcrit
