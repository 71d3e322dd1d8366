"""GPU parity of the Jacobi halo exchange (a persistent plan of row copies)
against the oracle: whole pools at a small grid over several replays, and
sampled rows at the paper's size (704^3 cells over 1 x 2 x 22 subgrids,
ghost layers two cells deep)."""
import numpy as np
import pytest

import oracle
from workloads import halo
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


def _rig(torch, H, ctx, N, Py, Pz, h):
    sb = halo.sub_bytes(N, Py, Pz, h)
    pool = torch.empty(Py * Pz * sb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + s * sb, sb)[1]
                      for s in range(Py * Pz)], dtype=np.uint32)
    d = halo.exchange(N, Py, Pz, h)
    dd = d.copy()
    dd["dst_slot"], dd["src_slot"] = slots[d["dst_slot"]], slots[d["src_slot"]]
    return pool, slots, d, dd, sb


def test_small_grid_plan_replays(env):
    torch, H, wd, ctx = env
    N, Py, Pz, h = 40, 2, 4, 2
    pool, slots, d, dd, sb = _rig(torch, H, ctx, N, Py, Pz, h)
    rc, plan, _ = H.hicr_plan_create(ctx, dd, H.hicr_sched_class(0)[1], H.PLAN_GRAPH)
    assert rc == H.OK, H.hicr_last_error(ctx)
    L = Py * Pz * sb
    for k in range(3):
        seed = 7100 + k
        _say("halo small replay", k)
        wd.fill(pool.data_ptr(), L, seed)
        torch.cuda.synchronize()
        assert H.hicr_plan_launch(plan) == H.OK
        assert H.hicr_fence(ctx) == H.OK
        host = content(seed, 0, L)
        oc = oracle.Ctx()
        ids = np.array([oc.register(host, offset=s * sb, size=sb)[1] for s in range(Py * Pz)])
        od = d.copy()
        od["dst_slot"], od["src_slot"] = ids[d["dst_slot"]], ids[d["src_slot"]]
        assert oc.memcpy_batch(od)[0] == oracle.OK
        assert np.array_equal(pool.cpu().numpy(), host), k
    assert H.hicr_plan_destroy(plan) == H.OK
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK


def test_full_size_sampled_rows(env):
    """704^3 over 1 x 2 x 22 subgrids, h = 2 (3.2 GB, 61,952 rows): one
    replay of the plan the benchmark times; 300 sampled rows and the cells
    around them are checked against the oracle's copy of each request."""
    torch, H, wd, ctx = env
    N, Py, Pz, h = 704, 2, 22, 2
    pool, slots, d, dd, sb = _rig(torch, H, ctx, N, Py, Pz, h)
    seed = 7200
    wd.fill(pool.data_ptr(), pool.numel(), seed)
    torch.cuda.synchronize()
    rc, plan, _ = H.hicr_plan_create(ctx, dd, H.hicr_sched_class(4)[1])
    assert rc == H.OK, H.hicr_last_error(ctx)
    _say("halo full replay")
    assert H.hicr_plan_launch(plan) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    g = np.random.default_rng(5)
    for i in g.choice(len(d), 300, replace=False):
        r = d[i]
        da = int(r["dst_slot"]) * sb + int(r["dst_off"])
        sa = int(r["src_slot"]) * sb + int(r["src_off"])
        n = int(r["size"])
        # one ghost cell on each side of the row is outside every request
        win = pool[da - 8:da + n + 8].cpu().numpy()
        want = content(seed, da - 8, n + 16)
        c = oracle.Ctx()
        _, w = c.register(want)
        _, s = c.register(content(seed, sa, n))
        assert c.memcpy(w, 8, s, 0, n) == oracle.OK
        assert np.array_equal(win, want), i
    assert sum(H.hicr_slot_counters(ctx, int(s))[2] for s in slots) == len(d)
    assert sum(H.hicr_slot_counters(ctx, int(s))[1] for s in slots) == len(d)
    assert H.hicr_plan_destroy(plan) == H.OK
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK
    del pool
    torch.cuda.empty_cache()


def test_reference_rows_kernel_copies_the_rows(env):
    """The benchmark's plain reference copy of the halo rows (measurement
    only) moves exactly the bytes the oracle moves, so its rate compares
    like with like."""
    torch, H, wd, ctx = env
    N, Py, Pz, h = 40, 2, 4, 2
    sb = halo.sub_bytes(N, Py, Pz, h)
    L = Py * Pz * sb
    pool = torch.empty(L, dtype=torch.uint8, device="cuda")
    seed = 7200
    wd.fill(pool.data_ptr(), L, seed)
    d = halo.exchange(N, Py, Pz, h)
    row = int(d["size"][0])
    base = np.uint64(pool.data_ptr())
    dst = torch.from_numpy((base + d["dst_slot"].astype(np.uint64) * np.uint64(sb)
                            + d["dst_off"]).view(np.int64)).to("cuda")
    src = torch.from_numpy((base + d["src_slot"].astype(np.uint64) * np.uint64(sb)
                            + d["src_off"]).view(np.int64)).to("cuda")
    torch.cuda.synchronize()
    _say("halo reference rows", len(d), row)
    wd.ref_rows(dst.data_ptr(), src.data_ptr(), len(d), row, 64)
    torch.cuda.synchronize()
    host = content(seed, 0, L)
    oc = oracle.Ctx()
    ids = np.array([oc.register(host, offset=s * sb, size=sb)[1] for s in range(Py * Pz)])
    od = d.copy()
    od["dst_slot"], od["src_slot"] = ids[d["dst_slot"]], ids[d["src_slot"]]
    assert oc.memcpy_batch(od)[0] == oracle.OK
    assert np.array_equal(pool.cpu().numpy(), host)
