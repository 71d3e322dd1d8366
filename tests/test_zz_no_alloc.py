"""GPU: the batch submission that allocates nothing (hicr_memcpy_batch_noalloc)
gives the same bytes and counters as hicr_memcpy_batch, and both equal the
CPU oracle.  Two calls in a row, the second smaller (and on another stream),
so a stale workspace from the first would show; rejections enqueue nothing."""
import numpy as np
import pytest

import oracle
from workloads import memcpy as wm
from workloads.content import content

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    assert torch.cuda.is_available()
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK, H.hicr_strerror(rc)
    yield torch, H, wd, ctx
    assert H.hicr_ctx_destroy(ctx) == H.OK


def _say(*a):
    print(*a, flush=True)


def _large_batch(seed):
    """8,193 requests of 0..256 KiB at odd offsets: more than 4,096, so the
    piece table is scanned into the workspace."""
    g = np.random.default_rng(seed)
    n = 8193
    sz = np.floor(np.exp(g.uniform(0, np.log(256 << 10), n))).astype(np.int64)
    sz[g.integers(0, n, 50)] = 0
    gap = g.integers(0, 200, n)
    dst = np.concatenate([[0], np.cumsum(sz + gap)[:-1]]) + 7
    src_base = int(dst[-1] + sz[-1] + 4096)
    src = src_base + np.concatenate([[0], np.cumsum(sz + gap[::-1])[:-1]]) + 11
    pool_len = int(src[-1] + sz[-1] + 64)
    d = np.zeros(n, dtype=wm.DESC_DTYPE)
    d["dst_slot"], d["src_slot"] = 0, 1
    d["dst_off"], d["src_off"], d["size"] = dst, src - src_base, sz
    return d, [0, src_base], [src_base, pool_len - src_base], pool_len


def _tiny_batch():
    bases, sizes, pool_len, descs, _ = wm.tiny(3)
    return descs, list(bases), list(sizes), pool_len


def _run_pair(env, descs, bases, sizes, pool_len, seed, sched, stream):
    """The same batch through both entry points on two pools filled alike;
    returns both pools' bytes and counters, and the oracle's."""
    torch, H, wd, ctx = env
    pools, slots = [], []
    for _ in range(2):
        p = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
        wd.fill(p.data_ptr(), pool_len, seed)
        sl = []
        for b, s in zip(bases, sizes):
            rc, x = H.hicr_slot_register(ctx, p.data_ptr() + int(b), int(s), H.MEM_HBM)
            assert rc == H.OK, H.hicr_last_error(ctx)
            sl.append(x)
        pools.append(p)
        slots.append(np.array(sl, dtype=np.uint32))
    torch.cuda.synchronize()
    d0, d1 = descs.copy(), descs.copy()
    for d, sl in ((d0, slots[0]), (d1, slots[1])):
        d["dst_slot"], d["src_slot"] = sl[descs["dst_slot"]], sl[descs["src_slot"]]
    rc, _ = H.hicr_memcpy_batch(ctx, d0, sched)
    assert rc == H.OK, H.hicr_last_error(ctx)
    rc, _ = H.hicr_memcpy_batch_noalloc(ctx, d1, sched, stream)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK
    got = [p.cpu().numpy() for p in pools]
    cnt = [[H.hicr_slot_counters(ctx, int(x))[1:] for x in sl] for sl in slots]
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    for b, s in zip(bases, sizes):
        assert oc.register(host, offset=int(b), size=int(s))[0] == oracle.OK
    assert oc.memcpy_batch(descs)[0] == oracle.OK
    ocnt = [tuple(oc.counters(k)[1:]) for k in range(len(bases))]
    return got, cnt, host, ocnt


def test_noalloc_equals_memcpy_batch_twice(env):
    torch, H, wd, ctx = env
    side = torch.cuda.Stream()
    cases = [("large", _large_batch(5), 31, H.hicr_sched_class(5)[1], 0),
             ("tiny", _tiny_batch(), 32, H.hicr_sched_class(0)[1], side.cuda_stream)]
    for name, (descs, bases, sizes, pool_len), seed, sched, stream in cases:
        _say("noalloc case", name, len(descs), pool_len)
        got, cnt, host, ocnt = _run_pair(env, descs, bases, sizes, pool_len, seed, sched, stream)
        assert np.array_equal(got[1], got[0]), name
        assert np.array_equal(got[0], host), name
        assert cnt[1] == cnt[0] == ocnt, name


def test_noalloc_rejections_enqueue_nothing(env):
    torch, H, wd, ctx = env
    n = 4096
    pool = torch.empty(2 * n, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), 2 * n, 9)
    torch.cuda.synchronize()
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), n, H.MEM_HBM)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + n, n, H.MEM_HBM)
    assert rc == rc2 == H.OK
    d = np.zeros(3, dtype=H.DESC_DTYPE)
    d["dst_slot"], d["src_slot"], d["size"] = a, b, 100
    d["dst_off"] = [0, 200, 400]
    d[2]["src_slot"] = 1 << 30  # no such slot
    _say("noalloc rejections")
    rc, bad = H.hicr_memcpy_batch_noalloc(ctx, d)
    assert rc == H.EBADSLOT and bad == 2
    too_many = np.zeros(65537, dtype=H.DESC_DTYPE)
    too_many["dst_slot"], too_many["src_slot"] = a, b
    assert H.hicr_memcpy_batch_noalloc(ctx, too_many)[0] == H.EINVAL
    learned = H.make_sched(64 << 10, 1, 2, H.SCHED_LEARNED)
    assert H.hicr_memcpy_batch_noalloc(ctx, d[:2], learned)[0] == H.EINVAL
    assert H.hicr_memcpy_batch_noalloc(ctx, d[:0])[0] == H.OK
    assert H.hicr_fence(ctx) == H.OK
    assert np.array_equal(pool.cpu().numpy(), content(9, 0, 2 * n))
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, 0)
    assert H.hicr_slot_counters(ctx, b) == (H.OK, 0, 0)
