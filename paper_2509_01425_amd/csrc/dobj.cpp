// dobj.cpp -- the data-object frontend (HiCR Sec. 4.3) over slots and memcpy.
//
// Publishing records {id, slot, offset, size} in the context and holds the
// slot; a get is one memcpy request from the object into the caller's slot,
// queued with the context's other single requests and moved by the fused
// copy kernel at the next fence.
#include <mutex>

#include "runtime.h"

using namespace hicr;

extern "C" {

int hicr_dobj_publish(hicr_ctx c, hicr_slot slot, uint64_t offset, uint64_t size,
                      uint64_t *id_out) {
  return guarded([&]() -> int {
    if (!c || !id_out) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    if (slot >= c->slots.size() || !c->slots[slot].live) return fail(c, HICR_EBADSLOT, "bad slot");
    Slot &s = c->slots[slot];
    if (size == 0 || offset > s.size || size > s.size - offset)
      return fail(c, HICR_ERANGE, "data object outside its slot");
    hicr_dobj_handle h{};
    h.id = c->next_dobj_id++;
    h.size = size;
    h.offset = offset;
    h.slot = slot;
    h.memspace = s.space;
    c->dobjs[h.id] = h;
    s.dobj_refs++;
    *id_out = h.id;
    return HICR_OK;
  });
}

int hicr_dobj_get_handle(hicr_ctx c, uint64_t id, hicr_dobj_handle *out) {
  return guarded([&]() -> int {
    if (!c || !out) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->dobjs.find(id);
    if (it == c->dobjs.end()) return fail(c, HICR_EINVAL, "no data object %llu", (unsigned long long)id);
    *out = it->second;
    return HICR_OK;
  });
}

int hicr_dobj_get(hicr_ctx c, const hicr_dobj_handle *h, hicr_slot dst, uint64_t dst_off) {
  return guarded([&]() -> int {
    if (!c || !h) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->dobjs.find(h->id);
    if (it == c->dobjs.end() || it->second.slot != h->slot || it->second.offset != h->offset ||
        it->second.size != h->size)
      return fail(c, HICR_EINVAL, "handle of a withdrawn data object");
    hicr_desc d{dst, h->slot, dst_off, h->offset, h->size};
    int rc = check_desc(c, d);
    if (rc != HICR_OK) return fail(c, rc, "data object get rejected");
    c->pending.push_back(d);
    if (c->pending.size() >= kMaxLdsDescs) {
      (void)hipSetDevice(c->device);
      return flush_pending(c);
    }
    return HICR_OK;
  });
}

int hicr_dobj_unpublish(hicr_ctx c, uint64_t id) {
  return guarded([&]() -> int {
    if (!c) return HICR_EINVAL;
    std::lock_guard<std::mutex> g(c->mu);
    auto it = c->dobjs.find(id);
    if (it == c->dobjs.end()) return fail(c, HICR_EINVAL, "no data object %llu", (unsigned long long)id);
    c->slots[it->second.slot].dobj_refs--;
    c->dobjs.erase(it);
    return HICR_OK;
  });
}

}  // extern "C"
