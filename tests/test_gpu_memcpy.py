"""GPU parity of the fused batched memcpy against the CPU oracle.

Every expected byte and counter comes from ``oracle`` on inputs drawn by
``workloads``; the comparison is bit-exact.
"""
import numpy as np
import pytest

import oracle
from tests.parity import abs_ranges, expected_window, oracle_counters, pmap
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


def _register_pool(H, ctx, pool, bases, sizes):
    slots = []
    for b, s in zip(bases, sizes):
        rc, sl = H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(s), H.MEM_HBM)
        assert rc == H.OK, H.hicr_last_error(ctx)
        slots.append(sl)
    return np.array(slots, dtype=np.uint32)


def _remap(descs, slots):
    d = descs.copy()
    d["dst_slot"] = slots[descs["dst_slot"]]
    d["src_slot"] = slots[descs["src_slot"]]
    return d


def test_device_fill_matches_generator(env):
    torch, H, wd, ctx = env
    for n, first in [(1, 0), (7, 8), (4096 + 5, 0), (1 << 20, 64), (3 << 20, 1 << 30)]:
        _say("fill", n, first)
        buf = torch.empty(n, dtype=torch.uint8, device="cuda")
        wd.fill(buf.data_ptr(), n, 77, first)
        torch.cuda.synchronize()
        assert np.array_equal(buf.cpu().numpy(), content(77, first, n))


@pytest.mark.parametrize("cls", list(range(12)))
def test_tiny_all_schedules(env, cls):
    """The tiny workload (64 packed slots, 256 requests) under every one of
    the 12 schedule classes: whole pool and every counter equal the oracle."""
    torch, H, wd, ctx = env
    bases, sizes, pool_len, descs, _ = wm.tiny(0)
    seed = 1000 + cls
    _say("tiny class", cls)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), pool_len, seed)
    torch.cuda.synchronize()
    slots = _register_pool(H, ctx, pool, bases, sizes)
    rc, sched = H.hicr_sched_class(cls)
    rc, bad = H.hicr_memcpy_batch(ctx, _remap(descs, slots), sched)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK
    got = pool.cpu().numpy()
    # oracle on the host
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    for b, s in zip(bases, sizes):
        assert oc.register(host, offset=int(b), size=int(s))[0] == oracle.OK
    assert oc.hazard_check(descs)[0] == oracle.OK
    assert oc.memcpy_batch(descs)[0] == oracle.OK
    assert np.array_equal(got, host), np.nonzero(got != host)[0][:10]
    for k, sl in enumerate(slots):
        rc, s, r = H.hicr_slot_counters(ctx, int(sl))
        assert (rc, s, r) == oc.counters(k)
    assert H.hicr_fence(ctx) == H.OK
    for sl in slots:
        assert H.hicr_slot_deregister(ctx, int(sl)) == H.OK


def test_alignment_grid_and_edges(env):
    """Every (dst mod 16, src mod 16) pair, sizes around 16/128/1K/64K piece
    edges, zero-size requests, one request spanning many pieces, under the
    smallest and largest chunk."""
    torch, H, wd, ctx = env
    g = np.random.default_rng(42)
    sizes = [0, 1, 2, 15, 16, 17, 31, 33, 127, 128, 129, 1023, 1025, 4095, 4097,
             65535, 65537, 200_003]
    reqs = []
    for da in range(16):
        for sa in range(16):
            reqs.append((da, sa, int(g.choice(sizes))))
    reqs.append((3, 9, (8 << 20) + 13))   # one large request: many pieces
    # lay requests out in one pool: destinations first, then sources
    cur = 0
    d_at, s_at = [], []
    for da, sa, n in reqs:
        cur = ((cur + 63) // 64) * 64 + da
        d_at.append(cur)
        cur += n + 16
    for da, sa, n in reqs:
        cur = ((cur + 63) // 64) * 64 + sa
        s_at.append(cur)
        cur += n + 16
    pool_len = cur + 64
    for cls in (0, 11):
        _say("alignment grid class", cls)
        seed = 500 + cls
        pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        rc, slot = H.hicr_slot_register(ctx, pool.data_ptr(), pool_len, H.MEM_HBM)
        assert rc == H.OK
        d = np.zeros(len(reqs), dtype=H.DESC_DTYPE)
        for i, (r, da, sa) in enumerate(zip(reqs, d_at, s_at)):
            d[i] = (slot, slot, da, sa, r[2])
        rc, sched = H.hicr_sched_class(cls)
        assert H.hicr_memcpy_batch(ctx, d, sched)[0] == H.OK
        assert H.hicr_fence(ctx) == H.OK
        host = content(seed, 0, pool_len)
        oc = oracle.Ctx()
        _, os_ = oc.register(host)
        od = d.copy()
        od["dst_slot"] = os_
        od["src_slot"] = os_
        assert oc.hazard_check(od)[0] == oracle.OK
        assert oc.memcpy_batch(od)[0] == oracle.OK
        got = pool.cpu().numpy()
        assert np.array_equal(got, host), np.nonzero(got != host)[0][:10]
        assert H.hicr_slot_counters(ctx, slot) == (H.OK, len(reqs), len(reqs))
        assert H.hicr_slot_deregister(ctx, slot) == H.OK


def test_many_requests_split_launches(env):
    """10,001 small requests: more than one 4,096-request launch."""
    torch, H, wd, ctx = env
    g = np.random.default_rng(3)
    n = 10_001
    sz = g.integers(0, 300, n)
    dst = np.concatenate([[0], np.cumsum(sz + 5)[:-1]]) + 3
    src_base = int(dst[-1] + sz[-1] + 4096)
    src = src_base + np.concatenate([[0], np.cumsum(sz + 1)[:-1]])
    pool_len = int(src[-1] + sz[-1] + 64)
    seed = 9
    _say("split launches", n)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), pool_len, seed)
    torch.cuda.synchronize()
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), src_base, H.MEM_HBM)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + src_base, pool_len - src_base, H.MEM_HBM)
    assert rc == rc2 == H.OK
    d = np.zeros(n, dtype=H.DESC_DTYPE)
    d["dst_slot"], d["src_slot"] = a, b
    d["dst_off"], d["src_off"], d["size"] = dst, src - src_base, sz
    rc, sched = H.hicr_sched_class(5)
    assert H.hicr_memcpy_batch(ctx, d, sched)[0] == H.OK
    assert H.hicr_fence(ctx) == H.OK
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    oa = oc.register(host, offset=0, size=src_base)[1]
    ob = oc.register(host, offset=src_base, size=pool_len - src_base)[1]
    od = d.copy()
    od["dst_slot"], od["src_slot"] = oa, ob
    assert oc.memcpy_batch(od)[0] == oracle.OK
    assert np.array_equal(pool.cpu().numpy(), host)
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, n)
    assert H.hicr_slot_counters(ctx, b) == (H.OK, n, 0)


def test_large_batch_scanned_table_all_classes(env):
    """8,193 requests of 0..256 KiB at odd offsets (more than 4,096, so the
    piece table is scanned once into device memory and every wavefront walks
    a range of it), under all 12 classes and as direct and graph plans."""
    torch, H, wd, ctx = env
    g = np.random.default_rng(5)
    n = 8193
    sz = np.floor(np.exp(g.uniform(0, np.log(256 << 10), n))).astype(np.int64)
    sz[g.integers(0, n, 50)] = 0
    gap = g.integers(0, 200, n)
    dst = np.concatenate([[0], np.cumsum(sz + gap)[:-1]]) + 7
    src_base = int(dst[-1] + sz[-1] + 4096)
    src = src_base + np.concatenate([[0], np.cumsum(sz + gap[::-1])[:-1]]) + 11
    pool_len = int(src[-1] + sz[-1] + 64)
    seed = 21
    _say("scanned table", n, pool_len)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), src_base, H.MEM_HBM)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + src_base, pool_len - src_base, H.MEM_HBM)
    assert rc == rc2 == H.OK
    d = np.zeros(n, dtype=H.DESC_DTYPE)
    d["dst_slot"], d["src_slot"] = a, b
    d["dst_off"], d["src_off"], d["size"] = dst, src - src_base, sz
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    oa = oc.register(host, offset=0, size=src_base)[1]
    ob = oc.register(host, offset=src_base, size=pool_len - src_base)[1]
    od = d.copy()
    od["dst_slot"], od["src_slot"] = oa, ob
    assert oc.memcpy_batch(od)[0] == oracle.OK
    runs = 0
    for cls in range(12):
        _say("scanned table class", cls)
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        assert H.hicr_memcpy_batch(ctx, d, H.hicr_sched_class(cls)[1])[0] == H.OK
        assert H.hicr_fence(ctx) == H.OK
        runs += 1
        assert np.array_equal(pool.cpu().numpy(), host), cls
    for flags in (0, H.PLAN_GRAPH):
        _say("scanned table plan flags", flags)
        rc, plan, _ = H.hicr_plan_create(ctx, d, H.hicr_sched_class(2)[1], flags)
        assert rc == H.OK, H.hicr_last_error(ctx)
        for _ in range(2):
            wd.fill(pool.data_ptr(), pool_len, seed)
            torch.cuda.synchronize()
            assert H.hicr_plan_launch(plan) == H.OK
            assert H.hicr_fence(ctx) == H.OK
            runs += 1
            assert np.array_equal(pool.cpu().numpy(), host), flags
        assert H.hicr_plan_destroy(plan) == H.OK
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, runs * n)
    assert H.hicr_slot_counters(ctx, b) == (H.OK, runs * n, 0)
    assert H.hicr_slot_deregister(ctx, a) == H.OK
    assert H.hicr_slot_deregister(ctx, b) == H.OK


def test_large_batch_threaded_checks_and_upload_stream(env):
    """24,000 requests: checked by several host threads and uploaded on the
    private stream.  Two bad requests (in different threads' parts): the
    lower index is reported and nothing moves.  Then the valid batch and a
    small batch right behind it on the same stream, the small one reading
    what the large one wrote, both against the oracle."""
    torch, H, wd, ctx = env
    n = 24_000
    g = np.random.default_rng(17)
    sz = g.integers(1, 600, n)
    dst = np.concatenate([[0], np.cumsum(sz + 3)[:-1]]) + 1
    src_base = int(dst[-1] + sz[-1] + 64)
    src = np.concatenate([[0], np.cumsum(sz + 5)[:-1]]) + 7
    tail_base = src_base + int(src[-1] + sz[-1] + 64)
    pool_len = tail_base + 4096
    seed = 31
    _say("threaded checks", n, pool_len)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), pool_len, seed)
    torch.cuda.synchronize()
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), src_base, H.MEM_HBM)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + src_base, pool_len - src_base, H.MEM_HBM)
    assert rc == rc2 == H.OK
    d = np.zeros(n, dtype=H.DESC_DTYPE)
    d["dst_slot"], d["src_slot"] = a, b
    d["dst_off"], d["src_off"], d["size"] = dst, src, sz
    bad = d.copy()
    bad[20_000]["size"] = src_base  # past the end of slot a
    bad[13_000]["src_slot"] = 999_999
    assert H.hicr_memcpy_batch(ctx, bad) == (H.EBADSLOT, 13_000)
    bad[13_000]["src_slot"] = b
    assert H.hicr_memcpy_batch(ctx, bad) == (H.ERANGE, 20_000)
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, 0)
    host = content(seed, 0, pool_len)
    assert np.array_equal(pool.cpu().numpy(), host)
    # the valid batch, then a small batch that copies part of its output
    small = np.zeros(4, dtype=H.DESC_DTYPE)
    small["dst_slot"], small["src_slot"] = b, a
    small["dst_off"] = tail_base - src_base + np.arange(4) * 1000
    small["src_off"] = dst[[0, 5000, 12_000, 23_000]]
    small["size"] = 900
    assert H.hicr_memcpy_batch(ctx, d, H.hicr_sched_class(5)[1])[0] == H.OK
    assert H.hicr_memcpy_batch(ctx, small, H.hicr_sched_class(5)[1])[0] == H.OK
    assert H.hicr_fence(ctx) == H.OK
    oc = oracle.Ctx()
    oa = oc.register(host, offset=0, size=src_base)[1]
    ob = oc.register(host, offset=src_base, size=pool_len - src_base)[1]
    for batch in (d, small):
        od = batch.copy()
        od["dst_slot"] = np.where(batch["dst_slot"] == a, oa, ob)
        od["src_slot"] = np.where(batch["src_slot"] == a, oa, ob)
        assert oc.memcpy_batch(od)[0] == oracle.OK
    assert np.array_equal(pool.cpu().numpy(), host)
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 4, n)
    assert H.hicr_slot_counters(ctx, b) == (H.OK, n, 4)
    assert H.hicr_slot_deregister(ctx, a) == H.OK
    assert H.hicr_slot_deregister(ctx, b) == H.OK


def test_concurrent_submitters_share_a_context(env):
    """Four host threads submit 40 batches each (and single memcpys) into one
    context at once, each into its own destination region; after one fence
    every byte and both slot counters match the oracle applying the same
    requests."""
    import threading
    torch, H, wd, ctx = env
    T, B, n = 4, 40, 64
    region = 1 << 20
    seed = 61
    pool_len = (T + 1) * region
    _say("concurrent submitters")
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), pool_len, seed)
    torch.cuda.synchronize()
    rc, dst = H.hicr_slot_register(ctx, pool.data_ptr(), T * region, H.MEM_HBM)
    rc2, src = H.hicr_slot_register(ctx, pool.data_ptr() + T * region, region, H.MEM_HBM)
    assert rc == rc2 == H.OK
    g = np.random.default_rng(12)
    work = []
    for t in range(T):
        batches = []
        for b in range(B):
            d = np.zeros(n, dtype=H.DESC_DTYPE)
            d["dst_slot"], d["src_slot"] = dst, src
            # request k of batch b writes its own 256-byte cell of the region
            d["dst_off"] = t * region + (b * n + np.arange(n)) * 256 + g.integers(0, 64, n)
            d["size"] = g.integers(0, 192, n)
            d["src_off"] = g.integers(0, region - 256, n)
            batches.append(d)
        work.append(batches)
    errors = []

    def run(t):
        try:
            for d in work[t]:
                assert H.hicr_memcpy_batch(ctx, d)[0] == H.OK
            d = work[t][0][:1]
            assert H.hicr_memcpy(ctx, dst, int(d["dst_off"][0]), src, int(d["src_off"][0]),
                                 int(d["size"][0])) == H.OK
        except AssertionError as e:
            errors.append(e)

    threads = [threading.Thread(target=run, args=(t,)) for t in range(T)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors
    assert H.hicr_fence(ctx) == H.OK
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    od_ = oc.register(host, offset=0, size=T * region)[1]
    os_ = oc.register(host, offset=T * region, size=region)[1]
    total = 0
    for t in range(T):
        for d in work[t] + [work[t][0][:1]]:
            od = d.copy()
            od["dst_slot"], od["src_slot"] = od_, os_
            assert oc.memcpy_batch(od)[0] == oracle.OK
            total += len(d)
    assert np.array_equal(pool.cpu().numpy(), host)
    assert oc.counters(od_) == (oracle.OK, 0, total)
    assert oc.counters(os_) == (oracle.OK, total, 0)
    assert H.hicr_slot_counters(ctx, dst) == (H.OK, 0, total)
    assert H.hicr_slot_counters(ctx, src) == (H.OK, total, 0)
    assert H.hicr_slot_deregister(ctx, dst) == H.OK
    assert H.hicr_slot_deregister(ctx, src) == H.OK


def test_single_memcpy_broadcast_and_fence_slot(env):
    """One message copied to many destinations with single memcpy calls and
    one fence (the paper's broadcast example, on one memory space)."""
    torch, H, wd, ctx = env
    msg_len, ndst = 1000, 37
    _say("broadcast")
    msg = torch.empty(msg_len + 5, dtype=torch.uint8, device="cuda")
    wd.fill(msg.data_ptr(), msg_len + 5, 5)
    dsts = torch.zeros(ndst, msg_len + 3, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc, sm = H.hicr_slot_register(ctx, msg.data_ptr() + 5, msg_len, H.MEM_HBM)
    assert rc == H.OK
    dslots = []
    for k in range(ndst):
        rc, s = H.hicr_slot_register(ctx, dsts[k].data_ptr() + 3, msg_len, H.MEM_HBM)
        assert rc == H.OK
        dslots.append(s)
        assert H.hicr_memcpy(ctx, s, 0, sm, 0, msg_len) == H.OK
    assert H.hicr_fence_slot(ctx, sm, ndst, 0, 10**9) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    want = content(5, 5, msg_len)
    got = dsts.cpu().numpy()
    for k in range(ndst):
        assert np.array_equal(got[k, 3:], want) and not got[k, :3].any()
    assert H.hicr_slot_counters(ctx, sm) == (H.OK, ndst, 0)
    assert H.hicr_fence_slot(ctx, sm, ndst + 1, 0, 10**6) == H.ETIMEDOUT
    assert H.hicr_fence_slot(ctx, dslots[0], 0, 1, 10**6) == H.OK


def test_fence_after_chained_small_batches(env):
    """A fence that returns once a small batch's counter kernel has raised its
    done word must still leave every byte and counter visible.  A chain of
    batches, each reading the region the previous one wrote, with 1 to 1,025
    requests (1,024 is the largest batch with one counter group), fences after
    one batch or after five (every submission buffer in flight), and every
    fifth batch written to pinned host memory (the event decides there).
    After every fence the pool is read on torch's stream and the counters on
    the library's counter stream, both compared with the oracle applying the
    same chain; then a plan of 600 requests replayed directly 40 times, with a
    fence after every 1 to 3 replays, keeps every counter at the number of
    replays queued."""
    torch, H, wd, ctx = env
    R, cell = 512 << 10, 256
    seed = 99
    _say("chained small batches")
    pool = torch.empty(3 * R, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), 3 * R, seed)
    torch.cuda.synchronize()
    hostbuf = torch.zeros(R, dtype=torch.uint8).pin_memory()
    rc, sp = H.hicr_slot_register(ctx, pool.data_ptr(), 3 * R, H.MEM_HBM)
    rc2, sh = H.hicr_slot_register(ctx, hostbuf.data_ptr(), R, H.MEM_HOST)
    assert rc == rc2 == H.OK
    want = content(seed, 0, 3 * R)
    want_h = np.zeros(R, dtype=np.uint8)
    oc = oracle.Ctx(pair_mask=0b1111)
    op = oc.register(want, offset=0, size=3 * R)[1]
    oh = oc.register(want_h, offset=0, size=R, space=oracle.MEM_HOST)[1]
    g = np.random.default_rng(7)
    sizes = [1, 7, 256, 1000, 1024, 1025, 64, 3]
    queued = 0
    for k in range(40):
        group = 5 if k % 7 == 3 else 1
        for j in range(group):
            it = k * 5 + j
            m = sizes[it % len(sizes)]
            to_host = it % 5 == 4
            src_r, dst_r = it % 3, (it + 1) % 3
            d = np.zeros(m, dtype=H.DESC_DTYPE)
            d["src_slot"] = sp
            d["src_off"] = src_r * R + g.integers(0, R - cell, m)
            cells = g.permutation(R // cell)[:m]
            d["size"] = g.integers(0, 200, m)
            off = cells * cell + g.integers(0, cell - 200, m)
            if to_host:
                d["dst_slot"], d["dst_off"] = sh, off
            else:
                d["dst_slot"], d["dst_off"] = sp, dst_r * R + off
            rc, bad = H.hicr_memcpy_batch(ctx, d)
            assert rc == H.OK, H.hicr_last_error(ctx)
            od = d.copy()
            od["src_slot"] = op
            od["dst_slot"] = oh if to_host else op
            assert oc.memcpy_batch(od)[0] == oracle.OK
            queued += m
        assert H.hicr_fence(ctx) == H.OK
        got = pool.cpu().numpy()
        assert np.array_equal(got, want), (k, np.nonzero(got != want)[0][:8])
        assert np.array_equal(hostbuf.numpy(), want_h), k
        assert H.hicr_slot_counters(ctx, sp)[1:] == oc.counters(op)[1:], k
        assert H.hicr_slot_counters(ctx, sh)[1:] == oc.counters(oh)[1:], k
    # a plan with one counter group replayed directly
    n = 600
    d = np.zeros(n, dtype=H.DESC_DTYPE)
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), R, H.MEM_HBM)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + R, R, H.MEM_HBM)
    assert rc == rc2 == H.OK
    d["dst_slot"], d["src_slot"] = b, a
    d["dst_off"] = g.permutation(R // cell)[:n] * cell
    d["src_off"] = g.integers(0, R - cell, n)
    d["size"] = g.integers(1, cell, n)
    rc, plan, _ = H.hicr_plan_create(ctx, d, None, 0)
    assert rc == H.OK, H.hicr_last_error(ctx)
    od = d.copy()
    od["dst_slot"], od["src_slot"] = op, op
    od["dst_off"] += R
    assert oc.memcpy_batch(od)[0] == oracle.OK
    replays = 0
    while replays < 40:
        for _ in range(1 + replays % 3):
            assert H.hicr_plan_launch(plan, 0) == H.OK
            replays += 1
        assert H.hicr_fence(ctx) == H.OK
        assert H.hicr_slot_counters(ctx, a) == (H.OK, replays * n, 0), replays
        assert H.hicr_slot_counters(ctx, b) == (H.OK, 0, replays * n), replays
        got = pool.cpu().numpy()
        assert np.array_equal(got, want), (replays, np.nonzero(got != want)[0][:8])
    assert H.hicr_plan_destroy(plan) == H.OK
    for sl in (a, b, sp, sh):
        assert H.hicr_slot_deregister(ctx, sl) == H.OK


def test_rejections_enqueue_nothing(env):
    torch, H, wd, ctx = env
    _say("rejections")
    a = torch.arange(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    h = torch.zeros(64, dtype=torch.uint8).pin_memory()
    torch.cuda.synchronize()
    assert H.hicr_slot_register(ctx, a.data_ptr(), 0, H.MEM_HBM)[0] == H.EINVAL
    assert H.hicr_slot_register(ctx, 0, 8, H.MEM_HBM)[0] == H.EINVAL
    assert H.hicr_slot_register(ctx, h.data_ptr(), 64, H.MEM_HBM)[0] == H.EINVAL
    assert H.hicr_slot_register(ctx, a.data_ptr(), 64, 9)[0] == H.EINVAL
    _, sa = H.hicr_slot_register(ctx, a.data_ptr(), 64, H.MEM_HBM)
    _, sb = H.hicr_slot_register(ctx, b.data_ptr(), 64, H.MEM_HBM)
    rc, sh = H.hicr_slot_register(ctx, h.data_ptr(), 64, H.MEM_HOST)
    assert rc == H.OK
    d = np.zeros(3, dtype=H.DESC_DTYPE)
    d[:] = [(sb, sa, 0, 0, 8), (sb, sa, 8, 60, 8), (sb, sa, 16, 0, 4)]
    assert H.hicr_memcpy_batch(ctx, d) == (H.ERANGE, 1)
    d[1] = (sh, sa, 0, 0, 4)
    assert H.hicr_ctx_set_pairs(ctx, H.PAIR(H.MEM_HBM, H.MEM_HBM)) == H.OK
    assert H.hicr_memcpy_batch(ctx, d) == (H.EUNSUPPORTED, 1)
    assert H.hicr_ctx_set_pairs(ctx, H.PAIRS_ALL) == H.OK
    d[1] = (sb, 12345, 0, 0, 4)
    assert H.hicr_memcpy_batch(ctx, d) == (H.EBADSLOT, 1)
    assert H.hicr_memcpy(ctx, sb, 0, sa, 2**64 - 1, 2) == H.ERANGE
    assert H.hicr_fence(ctx) == H.OK
    assert not b.cpu().numpy().any()
    assert H.hicr_slot_counters(ctx, sa) == (H.OK, 0, 0)
    bad = H.make_sched(100, 1, 2)
    assert H.hicr_memcpy_batch(ctx, d[:1], bad)[0] == H.EINVAL
    # deregistration waits for the fence
    d[1] = (sb, sa, 8, 8, 8)
    assert H.hicr_memcpy_batch(ctx, d)[0] == H.OK
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_slot_deregister(ctx, sa) == H.OK
    assert H.hicr_slot_counters(ctx, sa)[0] == H.EBADSLOT
    assert H.hicr_memcpy(ctx, sb, 0, sa, 0, 1) == H.EBADSLOT


def test_single_request_over_4gib(env):
    """One request of 4 GiB + 12,345 bytes at odd offsets (64-bit piece
    arithmetic: more than 2^32 bytes in one request, a million 4 KiB pieces
    under class 0), under classes 0 and 9; both ends and sampled windows of
    the destination, with margins, against the oracle."""
    torch, H, wd, ctx = env
    S = (4 << 30) + 12_345
    D = 3
    SRC = D + S + (1 << 20) + 5
    pool_len = SRC + S + 4096
    seed = 515
    _say("single request", S, pool_len)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    rc, sl = H.hicr_slot_register(ctx, pool.data_ptr(), pool_len, H.MEM_HBM)
    assert rc == H.OK
    d = np.zeros(1, dtype=H.DESC_DTYPE)
    d[0] = (sl, sl, D, SRC, S)
    dabs, sabs, size = np.array([D]), np.array([SRC]), np.array([S])
    g = np.random.default_rng(8)
    wins = [(0, 4096 + 64), (D + S - 4096, D + S + 64)] + \
        [(int(w), int(w) + 4096) for w in g.integers(D, D + S - 4096, 30)]
    for cls in (0, 9):
        _say("single request class", cls)
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        assert H.hicr_memcpy_batch(ctx, d, H.hicr_sched_class(cls)[1])[0] == H.OK
        assert H.hicr_fence(ctx) == H.OK
        for w0, w1 in wins:
            want = expected_window(dabs, sabs, size, w0, w1, seed)
            assert np.array_equal(pool[w0:w1].cpu().numpy(), want), (cls, w0)
    assert H.hicr_slot_counters(ctx, sl) == (H.OK, 2, 2)
    assert H.hicr_slot_deregister(ctx, sl) == H.OK
    del pool
    torch.cuda.empty_cache()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("sched_text", ["bench", "5"])
def test_batched_full_size_whole(env, sched_text):
    """One batch of the measured configuration (8,192 slot windows over a
    64 GiB + 64 MiB pool, 4,096 requests, ~22 GB) in exactly the launch the
    benchmark times (its fixed schedule and the library's default grid), and
    under class 5.  Every
    destination range, with 64 bytes of margin on each side, is compared
    with the oracle; so are at least 1 GiB of untouched bytes sampled from
    the gaps between destinations, and all 8,192 slot counters."""
    torch, H, wd, ctx = env
    seed = 4242
    bases, sizes = wm.batched_slots()
    _say("batched full size: alloc", wm.B_POOL)
    pool = torch.empty(wm.B_POOL, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), wm.B_POOL, seed)
    torch.cuda.synchronize()
    slots = _register_pool(H, ctx, pool, bases, sizes)
    descs = wm.batched(0)
    assert H.hicr_ctx_set_copy_grid(ctx, 0) == H.OK
    import bench
    sched = bench.parse_sched(H, bench.BATCHED_SCHED if sched_text == "bench" else sched_text)
    _say("batched full size: submit", sched_text)
    rc, bad = H.hicr_memcpy_batch(ctx, _remap(descs, slots), sched)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK
    dabs, sabs, size = abs_ranges(descs, bases)
    L = wm.B_POOL
    wins = [(max(0, int(a) - 64), min(L, int(a + z) + 64)) for a, z in zip(dabs, size)]
    # untouched bytes: 4 MiB windows (or whole gaps) between destinations
    order = np.argsort(dabs)
    ends = np.concatenate([[0], (dabs + size)[order]])
    starts = np.concatenate([dabs[order], [L]])
    gaps = [(int(a), int(b)) for a, b in zip(ends, starts) if b - a > 256]
    g = np.random.default_rng(1)
    gap_bytes = 0
    for k in g.permutation(len(gaps)):
        a, b = gaps[k]
        w = min(4 << 20, b - a - 128)
        w0 = int(g.integers(a + 64, b - 64 - w + 1))
        wins.append((w0, w0 + w))
        gap_bytes += w
        if gap_bytes >= 1 << 30:
            break
    assert gap_bytes >= 1 << 30
    covered = int(sum(b - a for a, b in wins))
    _say(f"batched full size: checking {len(wins)} windows, {covered / 1e9:.2f} GB")

    def check(win):
        w0, w1 = win
        want = expected_window(dabs, sabs, size, w0, w1, seed)
        return bool(np.array_equal(pool[w0:w1].cpu().numpy(), want))

    ok = pmap(check, wins)
    bad_w = [w for w, k in zip(wins, ok) if not k]
    assert not bad_w, ("windows differ from the oracle", bad_w[:4], len(bad_w))
    assert covered >= int(size.sum()) + (1 << 30)
    exp = oracle_counters(descs, len(slots))
    got = np.array([H.hicr_slot_counters(ctx, int(sl))[1:] for sl in slots], dtype=np.uint64)
    assert np.array_equal(got, exp)
    assert int(got[:, 0].sum()) == int(got[:, 1].sum()) == len(descs)
    for sl in slots:
        assert H.hicr_slot_deregister(ctx, int(sl)) == H.OK
    del pool
    torch.cuda.empty_cache()
