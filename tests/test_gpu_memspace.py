"""GPU parity of memcpy across memory spaces (HBM and pinned host memory)
against the oracle, whose pair mask allows every pair here.

The paper's broadcast example (one source, one memcpy per destination in
every memory space, then a fence) is run with single memcpy calls.
"""
import numpy as np
import pytest

import oracle
from workloads.content import content

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    yield torch, H, wd, ctx
    assert H.hicr_ctx_destroy(ctx) == H.OK


def _requests(g, n, dlen, slen, max_size):
    """n requests with disjoint destinations inside [0, dlen) and sources
    anywhere in [0, slen); unaligned offsets, sizes 0..max_size."""
    sz = g.integers(0, max_size + 1, n)
    sz[:3] = [0, 1, max_size]
    gap = g.integers(0, 40, n)
    ends = np.cumsum(gap + sz)
    assert ends[-1] <= dlen
    do = ends - sz
    so = (g.random(n) * (slen - sz + 1)).astype(np.int64)
    return do, so, sz


@pytest.mark.parametrize("pair", ["hbm<-host", "host<-hbm", "host<-host", "mixed"])
def test_pairs_bit_exact(env, pair):
    torch, H, wd, ctx = env
    g = np.random.default_rng({"hbm<-host": 1, "host<-hbm": 2, "host<-host": 3, "mixed": 4}[pair])
    L = 3 << 20
    seed_d, seed_h = 61, 62
    dev = torch.empty(L, dtype=torch.uint8, device="cuda")
    wd.fill(dev.data_ptr(), L, seed_d)
    host = torch.from_numpy(content(seed_h, 0, L)).pin_memory()
    torch.cuda.synchronize()
    _say("memspace", pair)
    # slot 0: device half A, 1: device half B, 2: host half A, 3: host half B
    half = L // 2
    regs = [(dev.data_ptr(), H.MEM_HBM), (dev.data_ptr() + half, H.MEM_HBM),
            (host.data_ptr(), H.MEM_HOST), (host.data_ptr() + half, H.MEM_HOST)]
    slots = []
    for p, sp in regs:
        rc, s = H.hicr_slot_register(ctx, p, half, sp)
        assert rc == H.OK, H.hicr_last_error(ctx)
        slots.append(s)
    # destinations in the A halves, sources in the B halves (hazard-free)
    route = {"hbm<-host": [(0, 3)], "host<-hbm": [(2, 1)], "host<-host": [(2, 3)],
             "mixed": [(0, 3), (2, 1), (0, 1), (2, 3)]}[pair]
    d = np.zeros(0, dtype=H.DESC_DTYPE)
    for k, (dk, sk) in enumerate(route):
        do, so, sz = _requests(g, 300 // len(route), half // len(route), half, 6000)
        part = np.zeros(len(sz), dtype=H.DESC_DTYPE)
        part["dst_slot"], part["src_slot"] = slots[dk], slots[sk]
        part["dst_off"] = do + k * (half // len(route))
        part["src_off"], part["size"] = so, sz
        d = np.concatenate([d, part])
    assert H.hicr_memcpy_batch(ctx, d, H.hicr_sched_class(4)[1])[0] == H.OK
    assert H.hicr_fence(ctx) == H.OK
    # oracle: the same four regions over host copies of the initial contents
    want_d, want_h = content(seed_d, 0, L), content(seed_h, 0, L)
    oc = oracle.Ctx(pair_mask=0b1111)
    ids = [oc.register(want_d, offset=0, size=half)[1],
           oc.register(want_d, offset=half, size=half)[1],
           oc.register(want_h, offset=0, size=half, space=oracle.MEM_HOST)[1],
           oc.register(want_h, offset=half, size=half, space=oracle.MEM_HOST)[1]]
    od = d.copy()
    inv = {s: i for i, s in enumerate(slots)}
    od["dst_slot"] = [ids[inv[int(s)]] for s in d["dst_slot"]]
    od["src_slot"] = [ids[inv[int(s)]] for s in d["src_slot"]]
    assert oc.memcpy_batch(od)[0] == oracle.OK
    assert np.array_equal(dev.cpu().numpy(), want_d)
    assert np.array_equal(host.numpy(), want_h)
    for i, s in enumerate(slots):
        assert H.hicr_slot_counters(ctx, s) == oc.counters(ids[i])
    for s in slots:
        assert H.hicr_slot_deregister(ctx, s) == H.OK


def test_broadcast_to_every_memory_space(env):
    """One 100,003-byte message in HBM to 6 HBM and 6 host destinations with
    single memcpy calls and one fence; the source's sent counter reaches 12."""
    torch, H, wd, ctx = env
    n = 100_003
    msg = torch.empty(n + 9, dtype=torch.uint8, device="cuda")
    wd.fill(msg.data_ptr(), n + 9, 71)
    dd = torch.zeros(6, n + 5, dtype=torch.uint8, device="cuda")
    hd = torch.zeros(6, n + 5, dtype=torch.uint8).pin_memory()
    torch.cuda.synchronize()
    rc, sm = H.hicr_slot_register(ctx, msg.data_ptr() + 9, n, H.MEM_HBM)
    assert rc == H.OK
    dst = []
    for k in range(6):
        dst.append(H.hicr_slot_register(ctx, dd[k].data_ptr() + (k % 5), n, H.MEM_HBM)[1])
        dst.append(H.hicr_slot_register(ctx, hd[k].data_ptr() + (k % 3), n, H.MEM_HOST)[1])
    for s in dst:
        assert H.hicr_memcpy(ctx, s, 0, sm, 0, n) == H.OK
    assert H.hicr_fence_slot(ctx, sm, len(dst), 0, 10**9) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    want = content(71, 9, n)
    gd, gh = dd.cpu().numpy(), hd.numpy()
    for k in range(6):
        assert np.array_equal(gd[k, k % 5:k % 5 + n], want)
        assert np.array_equal(gh[k, k % 3:k % 3 + n], want)
        assert not gd[k, :k % 5].any() and not gd[k, k % 5 + n:].any()
        assert not gh[k, :k % 3].any() and not gh[k, k % 3 + n:].any()
    for s in dst:
        assert H.hicr_slot_counters(ctx, s) == (H.OK, 0, 1)
        assert H.hicr_slot_deregister(ctx, s) == H.OK
    assert H.hicr_slot_deregister(ctx, sm) == H.OK


def test_pair_mask_and_host_registration(env):
    torch, H, wd, ctx = env
    a = torch.zeros(256, dtype=torch.uint8, device="cuda")
    h = torch.zeros(256, dtype=torch.uint8).pin_memory()
    pageable = np.zeros(256, np.uint8)
    torch.cuda.synchronize()
    assert H.hicr_slot_register(ctx, pageable.ctypes.data, 256, H.MEM_HOST)[0] == H.EINVAL
    assert H.hicr_slot_register(ctx, a.data_ptr(), 256, H.MEM_HOST)[0] == H.EINVAL
    assert H.hicr_slot_register(ctx, h.data_ptr(), 256, H.MEM_HBM)[0] == H.EINVAL
    _, sa = H.hicr_slot_register(ctx, a.data_ptr(), 256, H.MEM_HBM)
    rc, sh = H.hicr_slot_register(ctx, h.data_ptr(), 256, H.MEM_HOST)
    assert rc == H.OK
    assert H.hicr_ctx_set_pairs(ctx, 1 << 4) == H.EINVAL
    assert H.hicr_ctx_set_pairs(ctx, H.PAIR(H.MEM_HBM, H.MEM_HBM)) == H.OK
    assert H.hicr_memcpy(ctx, sh, 0, sa, 0, 4) == H.EUNSUPPORTED
    assert H.hicr_memcpy(ctx, sa, 0, sh, 0, 4) == H.EUNSUPPORTED
    d = np.zeros(2, dtype=H.DESC_DTYPE)
    d[:] = [(sa, sa, 0, 128, 8), (sa, sh, 0, 0, 4)]
    assert H.hicr_memcpy_batch(ctx, d) == (H.EUNSUPPORTED, 1)
    assert H.hicr_ctx_set_pairs(ctx, H.PAIR(H.MEM_HOST, H.MEM_HBM)) == H.OK
    assert H.hicr_memcpy(ctx, sh, 0, sa, 0, 4) == H.OK
    assert H.hicr_memcpy(ctx, sa, 0, sh, 0, 4) == H.EUNSUPPORTED
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_ctx_set_pairs(ctx, H.PAIRS_ALL) == H.OK
    assert H.hicr_slot_counters(ctx, sh) == (H.OK, 0, 1)
    assert H.hicr_slot_deregister(ctx, sa) == H.OK
    assert H.hicr_slot_deregister(ctx, sh) == H.OK
