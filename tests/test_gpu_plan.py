"""GPU parity of persistent batch plans (graph replays) against the oracle.

Each replay is checked on its own: between replays the pool is refilled
eagerly under a new seed (ordinary stream work and synchronisations between
graph launches), and the pool after the replay must equal the oracle's batch
applied to that seed's content; counters must equal k times the oracle's
counters after k replays.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from tests.parity import oracle_counters
from workloads import memcpy as wm
from workloads.content import content
from workloads.mlp_init import he_uniform

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


def _tiny_rig(torch, H, ctx, which=0):
    bases, sizes, pool_len, descs, _ = wm.tiny(which)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(s))[1]
                      for b, s in zip(bases, sizes)], dtype=np.uint32)
    d = descs.copy()
    d["dst_slot"], d["src_slot"] = slots[descs["dst_slot"]], slots[descs["src_slot"]]
    return bases, sizes, pool_len, descs, pool, slots, d


def _oracle_pool(bases, sizes, descs, seed, pool_len):
    host = content(seed, 0, pool_len)
    oc = oracle.Ctx()
    for b, s in zip(bases, sizes):
        oc.register(host, offset=int(b), size=int(s))
    assert oc.memcpy_batch(descs)[0] == oracle.OK
    return host


@pytest.mark.parametrize("cls,flags", [(0, 0), (5, 1), (11, 0), (11, 1)])
def test_tiny_plan_every_replay_matches_oracle(env, cls, flags):
    """Direct replay (flags 0) and graph replay (HICR_PLAN_GRAPH)."""
    torch, H, wd, ctx = env
    bases, sizes, pool_len, descs, pool, slots, d = _tiny_rig(torch, H, ctx)
    rc, plan, bad = H.hicr_plan_create(ctx, d, H.hicr_sched_class(cls)[1], flags)
    assert rc == H.OK, H.hicr_last_error(ctx)
    base_ctr = np.array([H.hicr_slot_counters(ctx, int(s))[1:] for s in slots], np.uint64)
    per = oracle_counters(descs, len(slots))
    for k in range(1, 6):
        seed = 3000 + 10 * cls + 100 * flags + k
        _say("plan replay", cls, k)
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        assert H.hicr_plan_launch(plan) == H.OK
        assert H.hicr_fence(ctx) == H.OK
        want = _oracle_pool(bases, sizes, descs, seed, pool_len)
        got = pool.cpu().numpy()
        assert np.array_equal(got, want), (k, np.nonzero(got != want)[0][:8])
        ctr = np.array([H.hicr_slot_counters(ctx, int(s))[1:] for s in slots], np.uint64)
        assert np.array_equal(ctr - base_ctr, per * np.uint64(k)), k
    # a slot a plan names cannot go away while the plan exists
    assert H.hicr_slot_deregister(ctx, int(slots[descs["dst_slot"][0]])) == H.EBUSY
    assert H.hicr_plan_destroy(plan) == H.OK
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK


@pytest.mark.parametrize("flags", [0, 1])
def test_plan_split_launches_and_stream_switch(env, flags):
    """10,001 requests (three copy launches), replayed alternately on two
    streams: each replay waits for the previous one."""
    torch, H, wd, ctx = env
    g = np.random.default_rng(8)
    n = 10_001
    sz = g.integers(0, 400, n)
    dst = np.concatenate([[0], np.cumsum(sz + 7)[:-1]]) + 5
    src_base = int(dst[-1] + sz[-1] + 4096)
    src = src_base + np.concatenate([[0], np.cumsum(sz + 3)[:-1]])
    pool_len = int(src[-1] + sz[-1] + 64)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc, a = H.hicr_slot_register(ctx, pool.data_ptr(), src_base)
    rc2, b = H.hicr_slot_register(ctx, pool.data_ptr() + src_base, pool_len - src_base)
    assert rc == rc2 == H.OK
    d = np.zeros(n, dtype=H.DESC_DTYPE)
    d["dst_slot"], d["src_slot"] = a, b
    d["dst_off"], d["src_off"], d["size"] = dst, src - src_base, sz
    rc, plan, _ = H.hicr_plan_create(ctx, d, H.hicr_sched_class(1)[1], flags)
    assert rc == H.OK, H.hicr_last_error(ctx)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    od = d.copy()
    for k in range(4):
        seed = 4100 + 10 * flags + k
        _say("split plan replay", k)
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        assert H.hicr_plan_launch(plan, (s1 if k % 2 else s2).cuda_stream) == H.OK
        assert H.hicr_fence(ctx) == H.OK
        host = content(seed, 0, pool_len)
        oc = oracle.Ctx()
        od["dst_slot"] = oc.register(host, offset=0, size=src_base)[1]
        od["src_slot"] = oc.register(host, offset=src_base, size=pool_len - src_base)[1]
        assert oc.memcpy_batch(od)[0] == oracle.OK
        assert np.array_equal(pool.cpu().numpy(), host), k
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, 4 * n)
    assert H.hicr_slot_counters(ctx, b) == (H.OK, 4 * n, 0)
    # back-to-back replays on two streams without a host wait in between:
    # the counters still count every replay exactly once
    for k in range(6):
        assert H.hicr_plan_launch(plan, (s1 if k % 2 else s2).cuda_stream) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_slot_counters(ctx, a) == (H.OK, 0, 10 * n)
    assert H.hicr_plan_destroy(plan) == H.OK
    assert H.hicr_slot_deregister(ctx, a) == H.OK
    assert H.hicr_slot_deregister(ctx, b) == H.OK


def test_plan_learned_choice_and_rejections(env):
    torch, H, wd, ctx = env
    bases, sizes, pool_len, descs, pool, slots, d = _tiny_rig(torch, H, ctx, 2)
    p = mlp.unpack(he_uniform(77).astype(np.float64))
    p["b3"][:] = 0
    p["b3"][9] = 20.0
    theta = mlp.pack(p).astype(np.float32)
    assert H.hicr_mlp_set_params(ctx, theta) == H.OK
    assert int(mlp.predict(theta.astype(np.float64), mlp.features(descs["size"]))[0]) == 9
    rc, plan, _ = H.hicr_plan_create(ctx, d, H.make_sched(65536, 1, 2, H.SCHED_LEARNED),
                                     H.PLAN_GRAPH)
    assert rc == H.OK, H.hicr_last_error(ctx)
    # a plan's class comes from the device forward kernel
    assert H.hicr_last_choice(ctx) == (H.OK, 9)
    for k in range(2):
        seed = 5200 + k
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        assert H.hicr_plan_launch(plan) == H.OK
        assert H.hicr_fence(ctx) == H.OK
        assert np.array_equal(pool.cpu().numpy(),
                              _oracle_pool(bases, sizes, descs, seed, pool_len)), k
    assert H.hicr_plan_destroy(plan) == H.OK
    # rejections: nothing is created
    bad = d.copy()
    bad["size"][17] = 1 << 40
    rc, plan, idx = H.hicr_plan_create(ctx, bad)
    assert (rc, plan, idx) == (H.ERANGE, None, 17)
    bad = d.copy()
    bad["src_slot"][3] = 10**6
    assert H.hicr_plan_create(ctx, bad)[0] == H.EBADSLOT
    assert H.hicr_plan_create(ctx, d, None, 2)[0] == H.EINVAL
    # an empty plan launches nothing
    rc, plan, _ = H.hicr_plan_create(ctx, d[:0])
    assert rc == H.OK
    assert H.hicr_plan_launch(plan) == H.OK
    assert H.hicr_plan_destroy(plan) == H.OK
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK


def test_plan_device_choice_equals_submission_choice(env):
    """A plan's class (device forward kernel) and a submission's class (host
    pass in the same arithmetic) agree on random networks and batches, except
    where the oracle's two best logits are within 1e-5 (relative)."""
    torch, H, wd, ctx = env
    bases, sizes, pool_len, descs, pool, slots, d = _tiny_rig(torch, H, ctx, 3)
    learned = H.make_sched(65536, 1, 2, H.SCHED_LEARNED)
    g = np.random.default_rng(12)
    agree = 0
    for trial in range(24):
        theta = he_uniform(300 + trial).astype(np.float32)
        p = mlp.unpack(theta.astype(np.float64))
        p["b3"][:] = g.normal(0, 0.5, 12)
        theta = mlp.pack(p).astype(np.float32)
        assert H.hicr_mlp_set_params(ctx, theta) == H.OK
        sub = d[g.permutation(len(d))[:int(g.integers(1, len(d) + 1))]]
        rc, plan, _ = H.hicr_plan_create(ctx, sub, learned)
        assert rc == H.OK, H.hicr_last_error(ctx)
        dev = H.hicr_last_choice(ctx)[1]
        assert H.hicr_plan_destroy(plan) == H.OK
        assert H.hicr_memcpy_batch(ctx, sub, learned)[0] == H.OK
        host = H.hicr_last_choice(ctx)[1]
        z = mlp.forward(theta.astype(np.float64), mlp.features(sub["size"])[None, :])[0][0]
        top = np.sort(z)[-2:]
        if abs(top[1] - top[0]) <= 1e-5 * max(abs(top[1]), 1e-30):
            continue
        assert dev == host == int(np.argmax(z)), trial
        agree += 1
    assert H.hicr_fence(ctx) == H.OK
    assert agree >= 20
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK
