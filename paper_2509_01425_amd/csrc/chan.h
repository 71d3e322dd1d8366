// chan.h -- ring-channel structures shared by the host runtime and the gfx950
// kernels (HiCR Sec. 4.3, Channels frontend).  Not part of the public ABI.
//
// A ring is a payload buffer of P bytes and an entry ring of E u64 entries,
// both in caller-registered HBM slots, plus a library-owned coordination
// block.  Counters are monotone: tm = messages published by the producer
// side, hm/hb = messages/bytes released by the consumer.  An entry is
// size | producer << 48.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hicr {

constexpr uint64_t kEntrySizeMask = (1ull << 48) - 1;
constexpr uint32_t kMaxProducers = 64;
constexpr int kPumpBlock = 256;
constexpr uint32_t kMaxTeam = 16;  // consumer workgroups of one locking MPSC ring

// One 128-byte line per writer so producer and consumer never share a line.
struct alignas(128) CoordLine {
  uint64_t w[16];
};

// Coordination block of one ring.
//   prod.w[0]  tm      messages published (producer side)
//   cons.w[0]  hm      messages released by the consumer
//   cons.w[1]  hb      bytes released by the consumer
//   lock.w[0]  ticket  next ticket (locking MPSC)
//   lock.w[1]  serving ticket allowed in
//   lock.w[2]  rm      messages reserved (locking MPSC, under the lock)
//   lock.w[3]  rb      bytes reserved     (locking MPSC, under the lock)
struct RingCoord {
  CoordLine prod;
  CoordLine cons;
  CoordLine lock;
};

struct DevRing {
  uint64_t payload;  // device address of P bytes
  uint64_t P;
  uint64_t entries;  // device address of E u64
  uint64_t E;
  uint64_t coord;    // device address of a RingCoord
  // locking MPSC rings in a pump: per-message records {absolute ring byte
  // position, output address, message index} indexed by (message counter -
  // base_m), written by the producer before it publishes
  uint64_t side;
  uint64_t base_m;   // the ring's message counter when the pump starts
  uint64_t side_n;   // records in `side` (messages of this pump through the ring)
};

enum : uint32_t { kModeSpsc = 0, kModeMpscLock = 1, kModeMpscNoLock = 2 };

// One consumer unit (one workgroup).  kModeMpscLock: a member of the team
// that consumes the shared ring of a locking MPSC channel (K producers told
// apart by the entry's producer tag); the team shares a claim counter and a
// round table (rounds[k] = end + 1 of round k once defined, 0 before).
// kModeSpsc: n_rings independent rings, each with exactly one producer stream
// (SPSC rings and non-locking MPSC sub-rings, possibly of different
// channels); ring q belongs to stream stream_of_prod[prod_stream_base + q].
struct DevChannel {
  uint32_t mode;
  uint32_t n_rings;
  uint32_t first_ring;  // index into the ring table (the unit's rings are consecutive)
  uint32_t K;           // producers (== n_rings for independent rings)
  uint64_t total_msgs;  // messages the unit must take
  uint64_t trace_base;  // first trace slot (locking MPSC)
  uint32_t prod_stream_base;  // index into stream_of_prod: K entries
  uint32_t pad;
  uint64_t claim;   // locking team: device address of the round claim counter
  uint64_t rounds;  // locking team: device address of the round table
};

struct DevStream {
  uint32_t channel;
  uint32_t producer;
  uint32_t ring;       // ring the producer writes
  uint32_t pad;
  uint64_t src_base;   // device address of the source slot
  uint64_t out_base;   // device address of the output slot
  uint64_t first_msg;  // index into msg_off/msg_size
  uint64_t n_msgs;
  uint64_t out_bytes;  // bound of its output: the sum of the stream's message sizes,
                       // or the output slot's size when the tables are on the device
  uint64_t trace_base; // first trace slot of the stream (rings consumed on their own)
  uint64_t src_bytes;  // size of the source slot
};

// Per-workgroup role: kind 0 = up to four producer waves (ids = streams),
// kind 1 = one consumer unit (ids[0] = unit).
struct DevRole {
  uint32_t kind;
  uint32_t count;
  uint32_t ids[4];
};

struct PumpArgs {
  const DevRing *rings;
  const DevChannel *chans;
  const DevStream *streams;
  const uint32_t *stream_of_prod;
  const DevRole *roles;
  const uint64_t *msg_off;
  const uint64_t *msg_size;
  uint32_t *trace;     // nullable: stream index of each consumed message, per channel order
  uint64_t *ts_push;   // nullable: wall clock (100 MHz) when each message was published
  uint64_t *ts_pop;    // nullable: wall clock when each message was consumed
  uint32_t *err;       // err[0] error bits, err[1] abort request, err[4..5] address of
                       // the host's abort word (pinned; nonzero asks the pump to stop)
  uint64_t timeout_ticks;
};

// Host-API push: one message (or k tokens) into one ring.
struct PushArgs {
  DevRing ring;
  uint64_t src;        // device address of the payload
  uint64_t bytes;      // total bytes (k * T for tokens)
  uint64_t pos;        // ring byte position of the first byte (tb mod P)
  uint64_t first_entry;  // entry index of the first message (tm)
  uint32_t n_entries;  // messages written (k tokens or 1)
  uint32_t producer;
  uint64_t entry_bytes;  // size written in each entry
  uint64_t *publish;   // host-coherent published counter
  uint64_t publish_value;
};

enum : uint32_t { kErrTimeout = 1, kErrAbort = 2, kErrCorrupt = 4 };

hipError_t launch_pump(const PumpArgs &a, uint32_t n_wgs, hipStream_t stream);
hipError_t launch_push(const PushArgs &a, hipStream_t stream);
int pump_occupancy(int *wgs_per_cu);

}  // namespace hicr
