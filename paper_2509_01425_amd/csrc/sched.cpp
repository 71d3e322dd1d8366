// sched.cpp -- schedule selection for a batch (fixed / autotuned / learned).
#include "runtime.h"

namespace hicr {

struct SchedState {};

int choose_sched(hicr_ctx c, const hicr_desc *, uint64_t, uint32_t mode, hicr_sched *,
                 const DevSched **, hipStream_t) {
  return fail(c, HICR_EINVAL, "schedule mode %u is not available on this context", mode);
}

void destroy_sched(hicr_ctx c) {
  delete c->sched;
  c->sched = nullptr;
}

}  // namespace hicr
