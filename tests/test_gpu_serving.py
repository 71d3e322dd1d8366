"""GPU tests of the continuous-batching server: every request's result in
the mix equals the oracle's result for that request alone, and equals the
server's result when the request runs alone; a small arena forces queueing
without ever exceeding the budget."""
import numpy as np
import pytest

import oracle
from tests.parity import oracle_fifo_outputs
from workloads import serving as ws
from workloads.content import content

pytestmark = pytest.mark.gpu

SEED = 1234
SRC = 64 << 20
P, E, NCH = 64 << 10, 64, 16


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rig():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    src = torch.empty(SRC, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), SRC, SEED)
    payload = torch.zeros(NCH * P, dtype=torch.uint8, device="cuda")
    entries = torch.zeros(NCH * E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    _, ss = H.hicr_slot_register(ctx, src.data_ptr(), SRC)
    chans = []
    for c in range(NCH):
        _, ps = H.hicr_slot_register(ctx, payload.data_ptr() + c * P, P)
        _, es = H.hicr_slot_register(ctx, entries.data_ptr() + c * E * 8, E * 8)
        rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_DEVICE,
                                                               ps, es, capacity=P, entries=E))
        assert rc == H.OK
        chans.append(ch)
    yield torch, H, ctx, ss, chans, (src, payload, entries)
    for ch in chans:
        H.hicr_channel_destroy(ch)
    assert H.hicr_ctx_destroy(ctx) == H.OK


def _small_trace(rate, duration, batch, big=False):
    return ws.trace(duration_s=duration, rate=rate, src_bytes=SRC, n_channels=NCH, batch=batch,
                    copy_n=(8, 64), copy_size=(64, (1 << 20) if big else 256 << 10),
                    burst_m=(1, 32), burst_size=(16, 32 << 10))


def _expected(tr, q):
    """The oracle's result of request q run alone."""
    r = tr.reqs[q]
    f, n = int(r["first"]), int(r["count"])
    if r["kind"] == 0:
        out = np.zeros(int(r["hbm_bytes"]), np.uint8)
        mask = np.zeros(len(out), bool)
        c = oracle.Ctx()
        _, o = c.register(out)
        for d in tr.descs[f:f + n]:
            so, sz, do = int(d["src_off"]), int(d["size"]), int(d["dst_off"])
            s = content(SEED, so, sz)
            if sz:
                _, si = c.register(s)
                assert c.memcpy(o, do, si, 0, sz) == oracle.OK
            mask[do:do + sz] = True
        return out, mask
    msgs = [content(SEED, int(o), int(z)) for o, z in
            zip(tr.msg_src_off[f:f + n], tr.msg_size[f:f + n])]
    out = oracle_fifo_outputs(P, E, msgs)
    return out, np.ones(len(out), bool)


def _run(torch, H, ctx, ss, chans, tr, budget, streams=3, max_batch=32):
    arena = torch.zeros(budget, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    rc, aslot = H.hicr_slot_register(ctx, arena.data_ptr(), budget)
    assert rc == H.OK
    results = {}

    def done(q, off):
        results[q] = arena[off:off + int(tr.reqs[q]["hbm_bytes"])].cpu().numpy()

    admit = np.zeros(len(tr.reqs), np.uint64)
    fin = np.zeros(len(tr.reqs), np.uint64)
    rc, st = H.hicr_serve(ctx, tr.reqs, aslot, ss, tr.descs, tr.msg_src_off, tr.msg_size, chans,
                          streams=streams, max_batch_reqs=max_batch, on_complete=done,
                          admit_ns=admit, done_ns=fin)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_slot_deregister(ctx, aslot) == H.OK
    return results, st, admit, fin


def test_mix_equals_alone_and_oracle(rig):
    torch, H, ctx, ss, chans, _ = rig
    tr = _small_trace(rate=40000, duration=0.01, batch=1)
    n = len(tr.reqs)
    _say("serving mix", n, "requests")
    res, st, admit, fin = _run(torch, H, ctx, ss, chans, tr, budget=256 << 20)
    assert st.completed == n and len(res) == n
    assert st.max_inflight_requests > 1           # work overlapped on the device
    for q in range(n):
        want, mask = _expected(tr, q)
        assert np.array_equal(res[q][mask], want[mask]), q
    # the same requests alone
    g = np.random.default_rng(0)
    for q in g.choice(n, 12, replace=False):
        one = tr.reqs[q:q + 1].copy()
        one["arrival_ns"] = 0
        alone, _, _, _ = _run(torch, H, ctx, ss, chans,
                              ws.Trace(one, tr.descs, tr.msg_src_off, tr.msg_size), 64 << 20)
        _, mask = _expected(tr, q)
        assert np.array_equal(alone[0][mask], res[q][mask])
    assert (fin >= admit).all()


def test_small_budget_forces_queueing(rig):
    torch, H, ctx, ss, chans, _ = rig
    tr = _small_trace(rate=20000, duration=0.01, batch=2, big=True)
    n = len(tr.reqs)
    budget = 3 * int(tr.reqs["hbm_bytes"].max()) + 4096
    _say("serving queueing", n, "requests, budget", budget)
    res, st, admit, fin = _run(torch, H, ctx, ss, chans, tr, budget=budget, streams=2)
    assert st.completed == n
    assert st.peak_arena_bytes <= budget
    wait = admit.astype(np.int64) - tr.reqs["arrival_ns"].astype(np.int64)
    assert (wait >= 0).all() and (wait > 200_000).sum() > n // 10   # many waited > 0.2 ms
    for q in range(0, n, 3):
        want, mask = _expected(tr, q)
        assert np.array_equal(res[q][mask], want[mask]), q


def test_serve_rejections(rig):
    torch, H, ctx, ss, chans, _ = rig
    tr = _small_trace(rate=1000, duration=0.01, batch=3)
    arena = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    _, aslot = H.hicr_slot_register(ctx, arena.data_ptr(), 1 << 20)
    big = tr.reqs.copy()
    big["hbm_bytes"][0] = 2 << 20
    assert H.hicr_serve(ctx, big, aslot, ss, tr.descs, tr.msg_src_off, tr.msg_size,
                        chans)[0] == H.ERANGE
    bad = tr.reqs.copy()
    if len(bad) > 1:
        bad["arrival_ns"][1] = 0
        bad["arrival_ns"][0] = 10
        assert H.hicr_serve(ctx, bad, aslot, ss, tr.descs, tr.msg_src_off, tr.msg_size,
                            chans)[0] == H.EINVAL
    assert H.hicr_slot_deregister(ctx, aslot) == H.OK
