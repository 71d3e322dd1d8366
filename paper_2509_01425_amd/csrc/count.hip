// count.hip -- per-slot transfer counters of a fused memcpy submission
// (HiCR Sec. 3.1.4: a slot counts its completed outgoing and incoming
// transfers).  count_kernel is queued on the submission's stream behind its
// copy launches, so every counted transfer's bytes are visible before its
// counters rise.
#include "internal.h"

namespace hicr {

// Raise sent (source) and received (destination) of every request's slots.
// Workgroup g takes requests [1024 g, 1024 g + 1024).  Requests often share
// slots (a halo exchange names 8 slots 28,160 times), and device atomics on
// one address serialise, so the counts are summed per slot in an LDS table
// first: a bucket holds one slot and a packed count (sent in bits 0..15,
// received in 16..31 -- at most 1,024 requests per group); a slot whose
// bucket another slot holds goes straight to device memory.  Slot ids are
// below 2^20, never ~0u.
// done != null (one-group launches only): once every wave's counter
// atomics have completed, the group stores seq to *done (host memory) at
// system scope, so that a host waiting for the submission can see its end
// without waiting for the runtime's completion signal.
__global__ __launch_bounds__(kCopyBlock) void count_kernel(const uint64_t *slots, uint64_t n,
                                                           uint64_t *counters, uint64_t *done,
                                                           uint64_t seq) {
  constexpr uint32_t kBuckets = 2048;
  constexpr uint32_t kPerGroup = 1024;  // requests per group: short serial chains
  constexpr uint32_t kEmpty = 0xffffffffu;
  __shared__ uint32_t key[kBuckets], cnt[kBuckets];
  const uint32_t tid = threadIdx.x;
  const uint64_t i0 = (uint64_t)blockIdx.x * kPerGroup;
  const uint64_t i1 = i0 + kPerGroup < n ? i0 + kPerGroup : n;
  for (uint32_t h = tid; h < kBuckets; h += kCopyBlock) {
    key[h] = kEmpty;
    cnt[h] = 0;
  }
  __syncthreads();
  // which: 0 = sent (low half of the packed count), 1 = received (high half)
  auto add = [&](uint32_t slot, uint32_t n_req, uint32_t which) {
    const uint32_t h = slot & (kBuckets - 1);
    const uint32_t old = atomicCAS(&key[h], kEmpty, slot);
    if (old == kEmpty || old == slot)
      atomicAdd(&cnt[h], n_req << (16 * which));
    else
      __hip_atomic_fetch_add(&counters[2 * (uint64_t)slot + which], (uint64_t)n_req,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // Each thread takes a contiguous run of requests and merges neighbours that
  // name the same slot before touching the table: batches list requests of
  // one slot together (the rows of one halo face), and LDS atomics on one
  // address from many lanes serialise too.
  const uint32_t per = (uint32_t)((i1 - i0 + kCopyBlock - 1) / kCopyBlock);
  const uint64_t r0 = i0 + (uint64_t)tid * per;
  const uint64_t r1 = r0 + per < i1 ? r0 + per : i1;
  uint32_t cur_s = kEmpty, cur_d = kEmpty, run_s = 0, run_d = 0;
  for (uint64_t i = r0; i < r1; i++) {
    const uint64_t sp = slots[i];
    const uint32_t dslot = (uint32_t)(sp & 0xffffffffull), sslot = (uint32_t)(sp >> 32);
    if (sslot != cur_s) {
      if (run_s) add(cur_s, run_s, 0);
      cur_s = sslot;
      run_s = 0;
    }
    if (dslot != cur_d) {
      if (run_d) add(cur_d, run_d, 1);
      cur_d = dslot;
      run_d = 0;
    }
    run_s++;
    run_d++;
  }
  if (run_s) add(cur_s, run_s, 0);
  if (run_d) add(cur_d, run_d, 1);
  __syncthreads();
  for (uint32_t h = tid; h < kBuckets; h += kCopyBlock) {
    const uint32_t k = key[h];
    if (k == kEmpty) continue;
    const uint32_t c = cnt[h];
    if (c & 0xffffu)
      __hip_atomic_fetch_add(&counters[2 * (uint64_t)k], (uint64_t)(c & 0xffffu),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c >> 16)
      __hip_atomic_fetch_add(&counters[2 * (uint64_t)k + 1], (uint64_t)(c >> 16),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (done) {
    // each wave's release orders its own atomics before the barrier; the
    // store's system-scope release then carries them all to the host
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(done, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

hipError_t launch_count(const uint64_t *slots, uint64_t n, uint64_t *counters, hipStream_t stream,
                        uint64_t *done, uint64_t seq, bool *armed) {
  if (armed) *armed = false;
  if (n == 0) return hipSuccess;
  const uint64_t groups = (n + 1023) / 1024;
  if (groups > 0x7fffffffull) return hipErrorInvalidValue;
  uint64_t *d = groups == 1 ? done : nullptr;
  hipLaunchKernelGGL(count_kernel, dim3((uint32_t)groups), dim3(kCopyBlock), 0, stream, slots, n,
                     counters, d, seq);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && armed) *armed = d != nullptr;
  return e;
}

}  // namespace hicr
