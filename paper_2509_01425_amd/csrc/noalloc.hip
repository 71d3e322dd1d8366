// noalloc.hip -- the fixed device workspace of hicr_memcpy_batch_noalloc.
//
// The workspace is a file-scope device array: every GPU the library runs on
// holds its own copy from module load until the process ends, so a
// submission through it never allocates device memory.  In host code the
// array's name only stands for the symbol; its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and that
// address is what every launch, copy and fill uses.
#include <mutex>

#include "noalloc.h"

namespace hicr {

// Packed requests (32 B each) followed by their piece tables (8 B each), for
// at most kNoAllocMaxReqs requests: the layout batch_bytes()/batch_tables()
// describe for any submission buffer.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices];
}  // namespace

hipError_t noalloc_scratch(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace hicr
