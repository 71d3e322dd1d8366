"""GPU parity of the data-object frontend: objects published from an HBM
slot, their identifiers sent through a fixed-size SPSC channel, fetched with
get into HBM and pinned-host slots; bytes and counters equal the oracle's
memcpy of each object."""
import numpy as np
import pytest

import oracle
from workloads.content import content

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    yield torch, H, wd, ctx
    assert H.hicr_ctx_destroy(ctx) == H.OK


def test_publish_send_id_get(env):
    torch, H, wd, ctx = env
    L, seed = 4 << 20, 81
    src = torch.empty(L, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), L, seed)
    dev_dst = torch.zeros(L, dtype=torch.uint8, device="cuda")
    host_dst = torch.zeros(L, dtype=torch.uint8).pin_memory()
    ids = torch.zeros(8, dtype=torch.int64, device="cuda")
    ring = torch.zeros(4 * 8, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(4, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    reg = lambda t, sp=H.MEM_HBM: H.hicr_slot_register(ctx, t.data_ptr(), t.numel() * t.element_size(), sp)[1]  # noqa: E731
    ss, sd, sh = reg(src), reg(dev_dst), reg(host_dst, H.MEM_HOST)
    s_ids, rs, es = reg(ids), reg(ring), reg(ent)
    objs = [(3, 1), (4096 + 5, 4097), (1 << 20, (1 << 20) + 3), (L - 77, 77)]
    published = []
    for off, n in objs:
        rc, oid = H.hicr_dobj_publish(ctx, ss, off, n)
        assert rc == H.OK
        published.append(oid)
    assert len(set(published)) == len(published)
    # the identifiers travel through a host-endpoint fixed SPSC channel of 8-byte tokens
    ids.copy_(torch.tensor(published + [0] * (8 - len(published)), dtype=torch.int64))
    torch.cuda.synchronize()
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_FIXED, H.CH_SPSC, 1, H.CH_HOST,
                                                           rs, es, token_bytes=8, capacity=4))
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_channel_push(ch, 0, s_ids, 0, len(objs)) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    received = []
    for i in range(len(objs)):
        rc, roff, size, _ = H.hicr_channel_peek(ch, 0, i)
        assert rc == H.OK and size == 8
        received.append(int(ring[roff:roff + 8].cpu().numpy().view(np.int64)[0]))
    assert H.hicr_channel_pop(ch, 0, len(objs)) == H.OK
    assert received == published
    # get every object into both destinations, at offsets of its own
    host = content(seed, 0, L)
    want_d, want_h = np.zeros(L, np.uint8), np.zeros(L, np.uint8)
    oc = oracle.Ctx(pair_mask=0b1111)
    _, o_src = oc.register(host)
    _, o_d = oc.register(want_d)
    _, o_h = oc.register(want_h, space=oracle.MEM_HOST)
    at = 0
    for oid in received:
        rc, h = H.hicr_dobj_get_handle(ctx, oid)
        assert rc == H.OK and h.slot == ss and h.memspace == H.MEM_HBM
        assert H.hicr_dobj_get(ctx, h, sd, at) == H.OK
        assert H.hicr_dobj_get(ctx, h, sh, at + 1) == H.OK
        assert oc.memcpy(o_d, at, o_src, h.offset, h.size) == oracle.OK
        assert oc.memcpy(o_h, at + 1, o_src, h.offset, h.size) == oracle.OK
        at += h.size + 64
    assert H.hicr_fence(ctx) == H.OK
    assert np.array_equal(dev_dst.cpu().numpy(), want_d)
    assert np.array_equal(host_dst.numpy(), want_h)
    assert H.hicr_slot_counters(ctx, ss) == (H.OK, 2 * len(objs), 0)
    assert H.hicr_slot_counters(ctx, sd) == (H.OK, 0, len(objs))
    assert H.hicr_slot_counters(ctx, sh) == (H.OK, 0, len(objs))
    # withdrawal
    assert H.hicr_slot_deregister(ctx, ss) == H.EBUSY
    rc, h0 = H.hicr_dobj_get_handle(ctx, published[0])
    for oid in published:
        assert H.hicr_dobj_unpublish(ctx, oid) == H.OK
    assert H.hicr_dobj_unpublish(ctx, published[0]) == H.EINVAL
    assert H.hicr_dobj_get_handle(ctx, published[0])[0] == H.EINVAL
    assert H.hicr_dobj_get(ctx, h0, sd, 0) == H.EINVAL
    rc, again = H.hicr_dobj_publish(ctx, ss, 0, 16)
    assert rc == H.OK and again not in published          # identifiers are never reused
    assert H.hicr_dobj_unpublish(ctx, again) == H.OK
    assert H.hicr_channel_destroy(ch) == H.OK
    for s in (ss, sd, sh, s_ids, rs, es):
        assert H.hicr_slot_deregister(ctx, s) == H.OK


def test_publish_rejections(env):
    torch, H, wd, ctx = env
    a = torch.zeros(100, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    _, sa = H.hicr_slot_register(ctx, a.data_ptr(), 100)
    assert H.hicr_dobj_publish(ctx, sa, 0, 0)[0] == H.ERANGE
    assert H.hicr_dobj_publish(ctx, sa, 90, 11)[0] == H.ERANGE
    assert H.hicr_dobj_publish(ctx, sa, 2**64 - 1, 2)[0] == H.ERANGE
    assert H.hicr_dobj_publish(ctx, 10**6, 0, 1)[0] == H.EBADSLOT
    assert H.hicr_dobj_get_handle(ctx, 10**12)[0] == H.EINVAL
    rc, oid = H.hicr_dobj_publish(ctx, sa, 10, 90)
    assert rc == H.OK
    rc, h = H.hicr_dobj_get_handle(ctx, oid)
    assert H.hicr_dobj_get(ctx, h, sa, 11) == H.ERANGE     # 11 + 90 > 100
    assert H.hicr_dobj_unpublish(ctx, oid) == H.OK
    assert H.hicr_slot_deregister(ctx, sa) == H.OK
