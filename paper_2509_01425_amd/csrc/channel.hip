// channel.hip -- gfx950 kernels of the ring channels (HiCR Sec. 4.3).
//
// Protocol (per ring; counters monotone, see chan.h):
//   producer: wait until the consumer's released counters leave room for the
//             message (entries tm - hm < E, bytes tb - hb + s <= P), write the
//             payload at byte position tb mod P (split across the ring end),
//             write the entry, release fence, publish tm + 1;
//   consumer: acquire-read tm; while tm > hm read entry hm mod E and the
//             payload at hb mod P, then release fence and publish hb + s and
//             hm + 1 -- the notification that frees the producer's room.
// Locking MPSC: a ticket lock (FIFO-fair) guards the room check and the
// reservation of [rb, rb + s) / entry rm; the copy runs outside the lock and
// publication follows ticket order, so the shared ring holds one total order
// and never overflows.  Non-locking MPSC: one ring per producer; the
// consumer polls them round robin.
//
// pump_kernel is persistent: every workgroup is either four independent
// producer waves (one stream each) or one consumer (all four waves).  The
// host launches no more workgroups than the device holds at once, and every
// wait gives up after a no-progress time-out or on the abort word, so every
// wave exits.
#include "chan.h"

namespace hicr {

#define GLOBAL __attribute__((address_space(1)))
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef v4u v4u_any __attribute__((aligned(1)));

constexpr uint32_t kBatch = 8;  // messages a consumer takes per notification

__device__ __forceinline__ uint64_t ld_acq(uint64_t a) {
  return __hip_atomic_load((uint64_t *)a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_rlx(uint64_t a) {
  return __hip_atomic_load((uint64_t *)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(uint64_t a, uint64_t v) {
  __hip_atomic_store((uint64_t *)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t a, uint64_t v) {
  __hip_atomic_store((uint64_t *)a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Copy n bytes d <- s with a team of TEAM threads (t = rank in the team):
// destination-aligned 16-byte stores, source at any alignment, at most 15
// head and 15 tail bytes one by one.  TEAM >= 64.
template <int TEAM, int U>
__device__ __forceinline__ void team_copy(uint64_t d, uint64_t s, uint64_t n, uint32_t t) {
  if (n == 0) return;
  uint64_t a0 = (d + 15) & ~(uint64_t)15;
  if (a0 > d + n) a0 = d + n;
  uint64_t a1 = (d + n) & ~(uint64_t)15;
  if (a1 < a0) a1 = a0;
  if (t < a0 - d) *(GLOBAL unsigned char *)(d + t) = *(const GLOBAL unsigned char *)(s + t);
  if (t >= 32 && t - 32 < d + n - a1) {
    uint64_t o = (a1 - d) + (t - 32);
    *(GLOBAL unsigned char *)(d + o) = *(const GLOBAL unsigned char *)(s + o);
  }
  const uint64_t nv = (a1 - a0) >> 4;
  const uint64_t s16 = s + (a0 - d);
  for (uint64_t b = 0; b < nv; b += (uint64_t)TEAM * U) {
    v4u r[U];
#pragma unroll
    for (int k = 0; k < U; k++) {
      uint64_t i = b + t + (uint64_t)k * TEAM;
      if (i < nv) r[k] = *(const GLOBAL v4u_any *)(s16 + 16 * i);
    }
#pragma unroll
    for (int k = 0; k < U; k++) {
      uint64_t i = b + t + (uint64_t)k * TEAM;
      if (i < nv) *(GLOBAL v4u *)(a0 + 16 * i) = r[k];
    }
  }
}

// Payload write / read at ring position pos, split across the ring end.
template <int TEAM, int U>
__device__ __forceinline__ void ring_put(const DevRing &r, uint64_t pos, uint64_t src, uint64_t n,
                                         uint32_t t) {
  uint64_t first = r.P - pos < n ? r.P - pos : n;
  team_copy<TEAM, U>(r.payload + pos, src, first, t);
  if (n > first) team_copy<TEAM, U>(r.payload, src + first, n - first, t);
}

template <int TEAM, int U>
__device__ __forceinline__ void ring_get(const DevRing &r, uint64_t pos, uint64_t dst, uint64_t n,
                                         uint32_t t) {
  uint64_t first = r.P - pos < n ? r.P - pos : n;
  team_copy<TEAM, U>(dst, r.payload + pos, first, t);
  if (n > first) team_copy<TEAM, U>(dst + first, r.payload, n - first, t);
}

// No-progress watchdog for spin waits.
struct Watch {
  uint64_t deadline, span;
  uint32_t *err;
  __device__ void progress() { deadline = wall_clock64() + span; }
  // true when the wait must stop (time-out recorded, or abort requested)
  __device__ bool expired() {
    if (__hip_atomic_load(&err[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
        __hip_atomic_load(&err[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
    if (wall_clock64() > deadline) {
      __hip_atomic_fetch_or(&err[0], kErrTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return true;
    }
    return false;
  }
};

__device__ __forceinline__ uint64_t wave_bcast(uint64_t v) {
  return ((uint64_t)__shfl((unsigned)(v >> 32), 0) << 32) | (uint64_t)__shfl((unsigned)v, 0);
}

// One producer wave drives one stream.
__device__ void run_producer(const PumpArgs &a, uint32_t sid, uint32_t lane) {
  const DevStream st = a.streams[sid];
  const DevRing r = a.rings[st.ring];
  const bool locking = a.chans[st.channel].mode == kModeMpscLock;
  const uint64_t c = r.coord;
  const uint64_t tm_a = c + offsetof(RingCoord, prod), hm_a = c + offsetof(RingCoord, cons),
                 hb_a = hm_a + 8, tk_a = c + offsetof(RingCoord, lock), sv_a = tk_a + 8,
                 rm_a = tk_a + 16, rb_a = tk_a + 24;
  // rings are empty when a pump starts: the producer side resumes at the
  // consumer's released counters
  uint64_t tm = ld_acq(tm_a), tb = ld_acq(hb_a);
  Watch w{0, a.timeout_ticks, a.err};
  w.progress();
  for (uint64_t m = 0; m < st.n_msgs; m++) {
    const uint64_t s = a.msg_size[st.first_msg + m];
    const uint64_t off = a.msg_off[st.first_msg + m];
    uint64_t my_tm = tm, my_tb = tb;
    if (locking) {
      uint64_t ticket = 0;
      if (lane == 0)
        ticket = __hip_atomic_fetch_add((uint64_t *)tk_a, 1ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
      ticket = wave_bcast(ticket);
      while (ld_acq(sv_a) != ticket) {
        __builtin_amdgcn_s_sleep(1);
        if (w.expired()) return;
      }
      my_tm = ld_rlx(rm_a);
      my_tb = ld_rlx(rb_a);
      while (!(my_tm - ld_acq(hm_a) < r.E && my_tb - ld_acq(hb_a) + s <= r.P)) {
        __builtin_amdgcn_s_sleep(2);
        if (w.expired()) return;
      }
      if (lane == 0) {
        st_rlx(rm_a, my_tm + 1);
        st_rlx(rb_a, my_tb + s);
        st_rel(sv_a, ticket + 1);
      }
    } else {
      while (!(my_tm - ld_acq(hm_a) < r.E && my_tb - ld_acq(hb_a) + s <= r.P)) {
        __builtin_amdgcn_s_sleep(2);
        if (w.expired()) return;
      }
    }
    ring_put<64, 4>(r, my_tb % r.P, st.src_base + off, s, lane);
    if (lane == 0)
      *(GLOBAL uint64_t *)(r.entries + 8 * (my_tm % r.E)) = s | ((uint64_t)st.producer << 48);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (locking) {
      while (ld_acq(tm_a) != my_tm) {  // publish in reservation order
        __builtin_amdgcn_s_sleep(1);
        if (w.expired()) return;
      }
    }
    if (lane == 0) {
      if (a.ts_push) a.ts_push[st.first_msg + m] = wall_clock64();
      st_rlx(tm_a, my_tm + 1);
    }
    tm = my_tm + 1;
    tb = my_tb + s;
    w.progress();
  }
}

// One consumer workgroup takes every message of one channel.
__device__ void run_consumer(const PumpArgs &a, uint32_t cid, uint32_t tid) {
  __shared__ uint64_t s_hm[kMaxProducers], s_hb[kMaxProducers];
  __shared__ uint64_t s_outpos[kMaxProducers], s_cnt[kMaxProducers];
  __shared__ uint64_t s_dst[kBatch], s_size[kBatch], s_pos[kBatch];
  __shared__ uint32_t s_ring, s_k, s_stop;
  const DevChannel ch = a.chans[cid];
  const uint32_t lane = tid & 63, wave = tid >> 6;
  for (uint32_t i = tid; i < ch.n_rings; i += kPumpBlock) {
    const uint64_t c = a.rings[ch.first_ring + i].coord + offsetof(RingCoord, cons);
    s_hm[i] = ld_acq(c);
    s_hb[i] = ld_acq(c + 8);
  }
  for (uint32_t p = tid; p < ch.K; p += kPumpBlock) {
    s_outpos[p] = 0;
    s_cnt[p] = 0;
  }
  __syncthreads();
  Watch w{0, a.timeout_ticks, a.err};
  w.progress();
  uint64_t done = 0;
  uint32_t rr = 0;
  while (done < ch.total_msgs) {
    if (wave == 0) {
      // lanes probe rings rr, rr+1, ... in parallel; take the first with data
      uint32_t ring = 0;
      uint64_t avail = 0;
      for (;;) {
        uint64_t av = 0;
        uint32_t ri = 0;
        if (lane < ch.n_rings) {
          ri = (rr + lane) % ch.n_rings;
          const uint64_t c = a.rings[ch.first_ring + ri].coord;
          av = ld_acq(c + offsetof(RingCoord, prod)) - s_hm[ri];
        }
        uint64_t m = __ballot(av > 0);
        if (m) {
          uint32_t f = (uint32_t)__ffsll((unsigned long long)m) - 1;
          ring = (uint32_t)__shfl((int)ri, (int)f);
          avail = ((uint64_t)__shfl((unsigned)(av >> 32), (int)f) << 32) |
                  (uint64_t)__shfl((unsigned)av, (int)f);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (w.expired()) {
          ring = ~0u;
          break;
        }
      }
      if (lane == 0) {
        const uint64_t left = ch.total_msgs - done;
        uint64_t k = avail < kBatch ? avail : kBatch;
        if (k > left) k = left;
        s_stop = ring == ~0u;
        s_ring = ring;
        s_k = (uint32_t)k;
      }
    }
    __syncthreads();
    if (s_stop) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const uint32_t ri = s_ring, k = s_k;
    const DevRing r = a.rings[ch.first_ring + ri];
    if (tid == 0) {
      // entries are checked against the plan before any byte moves: a
      // malformed entry stops the pump instead of writing out of bounds
      uint64_t pos = s_hb[ri] % r.P;
      uint32_t bad = 0;
      for (uint32_t i = 0; i < k; i++) {
        const uint64_t e = *(const GLOBAL uint64_t *)(r.entries + 8 * ((s_hm[ri] + i) % r.E));
        const uint64_t sz = e & kEntrySizeMask;
        const uint32_t p = (uint32_t)(e >> 48) % ch.K;
        const uint32_t sid = a.stream_of_prod[ch.prod_stream_base + p];
        const DevStream &so = a.streams[sid];
        if (sz > r.P || s_outpos[p] + sz > so.out_bytes || s_cnt[p] >= so.n_msgs) {
          bad = 1;
          s_size[i] = 0;
          continue;
        }
        s_dst[i] = so.out_base + s_outpos[p];
        s_size[i] = sz;
        s_pos[i] = pos;
        pos = (pos + sz) % r.P;
        s_outpos[p] += sz;
        if (a.trace) a.trace[ch.trace_base + done + i] = sid;
        if (a.ts_pop) a.ts_pop[so.first_msg + s_cnt[p]] = wall_clock64();
        s_cnt[p] += 1;
      }
      if (bad) {
        __hip_atomic_fetch_or(&a.err[0], kErrCorrupt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_stop = 1;
      }
    }
    __syncthreads();
    if (s_stop) break;
    uint64_t bytes = 0;
    for (uint32_t i = 0; i < k; i++) {
      ring_get<kPumpBlock, 4>(r, s_pos[i], s_dst[i], s_size[i], tid);
      bytes += s_size[i];
    }
    __syncthreads();  // every read of the ring has completed
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint64_t c = r.coord + offsetof(RingCoord, cons);
      st_rlx(c + 8, s_hb[ri] + bytes);
      st_rlx(c, s_hm[ri] + k);
      s_hm[ri] += k;
      s_hb[ri] += bytes;
    }
    done += k;
    rr = (ri + 1) % ch.n_rings;
    w.progress();
  }
  __threadfence();
}

__global__ __launch_bounds__(kPumpBlock) void pump_kernel(PumpArgs a) {
  const DevRole role = a.roles[blockIdx.x];
  const uint32_t tid = threadIdx.x;
  if (role.kind == 0) {
    const uint32_t wave = tid >> 6;
    if (wave < role.count) run_producer(a, role.ids[wave], tid & 63);
    __threadfence();
  } else {
    run_consumer(a, role.ids[0], tid);
  }
}

// Host-API push: copy the payload into the ring, write the entries, then
// publish the new message counter into host-coherent memory with a
// system-scope release.
__global__ __launch_bounds__(256) void push_kernel(PushArgs a) {
  const uint32_t tid = threadIdx.x;
  ring_put<256, 4>(a.ring, a.pos, a.src, a.bytes, tid);
  for (uint32_t i = tid; i < a.n_entries; i += 256)
    *(GLOBAL uint64_t *)(a.ring.entries + 8 * ((a.first_entry + i) % a.ring.E)) =
        a.entry_bytes | ((uint64_t)a.producer << 48);
  __threadfence_system();
  __syncthreads();
  if (tid == 0)
    __hip_atomic_store(a.publish, a.publish_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_pump(const PumpArgs &a, uint32_t n_wgs, hipStream_t stream) {
  hipLaunchKernelGGL(pump_kernel, dim3(n_wgs), dim3(kPumpBlock), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_push(const PushArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(push_kernel, dim3(1), dim3(256), 0, stream, a);
  return hipGetLastError();
}

int pump_occupancy(int *wgs_per_cu) {
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, pump_kernel, kPumpBlock, 0);
}

}  // namespace hicr
