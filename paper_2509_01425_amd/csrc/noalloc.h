// noalloc.h -- limits and workspace of the submission path that allocates
// nothing (hicr_memcpy_batch_noalloc).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hicr {

// Requests per call, and the device workspace they need: 32 B of packed
// request plus 8 B of piece tables each (2.5 MiB in all).
constexpr uint64_t kNoAllocMaxReqs = 65536;
constexpr uint64_t kNoAllocScratchBytes = kNoAllocMaxReqs * 40;
// Bytes per call: below this bound a batch of at most kNoAllocMaxReqs
// requests splits into at most three launches, so the launch list never
// outgrows the capacity reserved at context creation.
constexpr uint64_t kNoAllocMaxBytes = 1ull << 38;
constexpr size_t kNoAllocSegCap = 64;

// Device address of this device's workspace; `device` must be current.  The
// address is looked up on the first call for a device and kept.
hipError_t noalloc_scratch(int device, void **out);

}  // namespace hicr
