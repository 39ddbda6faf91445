// Static device scratch of ibmlbm_create_noalloc: for callers that cannot
// allocate device memory, every region of a solve other than its two lattice
// states (launch arguments, mass partials and flags, marker data, node-box
// images, force history) lives in this file-scope array, one copy per device,
// held until the process ends.  All such handles on one device share it.
#include <mutex>

#include "internal.h"

namespace ibmk {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's copy of `scratch`.  The array's name is a
// host-side stand-in in host code, so the address is looked up once per
// device, with that device current, and kept.
hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

}  // namespace ibmk
