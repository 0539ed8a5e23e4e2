// Fixed device scratch for the entry point that allocates nothing
// (mps_norm_noalloc): callers that cannot allocate device memory -- code
// under HIP graph capture, tight serving loops -- get the environment
// buffers of the norm's contraction from this static array instead of the
// handle's growable workspaces.
//
// Every GPU the library runs on holds its own copy of the array, at its own
// address, until the process ends.  Host code never passes the array's name
// to a kernel or a copy (in host code that name is a stand-in, not a device
// address): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that pointer is used
// everywhere.  All calls on one GPU share the array and leave the last call's
// contents behind; calls are serialised by scratch_lock() and each one
// finishes its device work before releasing it.
#include <mutex>
#include <vector>

#include "kernels.h"

namespace u1mps {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;              // guards g_scratch_ptr and every use of the arrays
std::vector<void*> g_scratch_ptr;     // per device: the array's device address
}  // namespace

std::unique_lock<std::mutex> scratch_lock() { return std::unique_lock<std::mutex>(g_scratch_mu); }

hipError_t scratch_region(int device, void** ptr, size_t* bytes) {
  // caller holds scratch_lock(), with `device` current
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  *bytes = kScratchBytes;
  return hipSuccess;
}

}  // namespace u1mps
