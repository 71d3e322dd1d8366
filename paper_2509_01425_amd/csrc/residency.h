// residency.h -- which earlier persistent launches a new one must follow.
//
// A channel pump is correct only while all of its workgroups are resident at
// once: a producer spins on a consumer of the same launch, and a consumer
// that is not yet dispatched waits for compute units that resident spinners
// never give back.  One launch is checked against the device on its own;
// launches in flight together on different streams must fit together too,
// and a ring may be driven by one launch at a time.  This is the admission
// rule, kept free of HIP so that it can be tested on the host.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace hicr {

struct LiveLaunch {
  uint64_t wgs;         // workgroups of the earlier launch
  bool done;            // its completion event has been observed
  bool same_stream;     // queued on the new launch's stream (so it ends first)
  bool shares_channel;  // drives a ring the new launch drives too
};

// Indices into `live` (oldest first) of the earlier launches the new one
// (new_wgs workgroups, on a device holding `cap` at once) must wait for:
// every unfinished one on another stream that shares a channel with it, then
// the oldest others until the ones left in flight fit beside it.  Launches
// already done or on the same stream are never waited for and never counted.
// When new_wgs <= cap, the waits leave at most cap - new_wgs workgroups of
// other launches possibly resident.
inline std::vector<size_t> residency_waits(const std::vector<LiveLaunch> &live, uint64_t new_wgs,
                                           uint64_t cap) {
  std::vector<size_t> waits;
  std::vector<bool> waited(live.size(), false);
  uint64_t others = 0;
  for (size_t i = 0; i < live.size(); i++) {
    const LiveLaunch &l = live[i];
    if (l.done || l.same_stream) continue;
    if (l.shares_channel) {
      waited[i] = true;
      continue;
    }
    others += l.wgs;
  }
  for (size_t i = 0; i < live.size(); i++) {
    const LiveLaunch &l = live[i];
    if (l.done || l.same_stream || waited[i]) continue;
    if (others + new_wgs <= cap) break;
    waited[i] = true;
    others -= l.wgs;
  }
  for (size_t i = 0; i < live.size(); i++)
    if (waited[i]) waits.push_back(i);
  return waits;
}

}  // namespace hicr
