"""GPU parity of the ring channels against the CPU oracle.

Host-API channels run in lock step with the oracle's rings (identical return
codes, offsets, sizes, producers and bytes).  Device pumps are checked per
stream against the outputs the oracle's rings produce for the same messages;
locking MPSC channels are checked by replaying the device's consumption
order through the oracle's shared ring (which also proves the order is a
merge of the producers' FIFO sequences).
"""
import numpy as np
import pytest

import oracle
from tests.parity import expected_stream_outputs, oracle_fifo_outputs, oracle_locking_outputs, pmap
from workloads import channels as wc
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


def _reg(H, ctx, t, off=0, size=None):
    size = t.numel() * t.element_size() - off if size is None else size
    rc, s = H.hicr_slot_register(ctx, t.data_ptr() + off, size, H.MEM_HBM)
    assert rc == H.OK, H.hicr_last_error(ctx)
    return s


def test_host_fixed_spsc_lockstep(env):
    """The tiny channel: 16 tokens x 256 B, 1,000 tokens, seeded attempts."""
    torch, H, wd, ctx = env
    C, T, N, seed = 16, 256, 1000, 31
    _say("host fixed spsc")
    src = torch.empty(N * T, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), N * T, seed)
    ring = torch.zeros(C * T, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(C, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ss, rs, es = _reg(H, ctx, src), _reg(H, ctx, ring), _reg(H, ctx, ent)
    cfg = H.make_channel_cfg(H.CH_FIXED, H.CH_SPSC, 1, H.CH_HOST, rs, es, token_bytes=T, capacity=C)
    rc, ch = H.hicr_channel_create(ctx, cfg)
    assert rc == H.OK, H.hicr_last_error(ctx)
    oc = oracle.FChan(C, T)
    host_src = content(seed, 0, N * T)
    sent = popped = 0
    n_eagain = 0
    for kind, k in wc.tiny_schedule() + [("pop", 1)] * (2 * N):
        if popped == N:
            break
        if kind == "push":
            k = min(k, N - sent)
            if k == 0:
                continue
            rc = H.hicr_channel_push(ch, 0, ss, sent * T, k)
            assert rc == oc.push(host_src[sent * T:], k)
            n_eagain += rc == H.EAGAIN
            if rc == H.OK:
                sent += k
                assert H.hicr_fence(ctx) == H.OK
        else:
            depth = oc.depth()
            assert H.hicr_channel_depth(ch, 0) == (H.OK, depth, depth * T)
            if depth:
                dev_ring = ring.cpu().numpy()
            for i in range(min(k, depth)):
                rc, off, sz, prod = H.hicr_channel_peek(ch, 0, i)
                ro, ooff = oc.peek(i)
                assert (rc, off, sz, prod) == (ro, ooff, T, 0)
                assert np.array_equal(dev_ring[off:off + T], oc.ring[ooff:ooff + T])
            if k > depth:
                assert H.hicr_channel_peek(ch, 0, depth)[0] == H.EAGAIN
            rc = H.hicr_channel_pop(ch, 0, k)
            assert rc == oc.pop(k)
            popped += k if rc == H.OK else 0
    assert popped == N and sent == N and n_eagain > 10
    # rejections
    assert H.hicr_channel_push(ch, 0, ss, 0, C + 1) == H.EINVAL
    assert H.hicr_channel_push(ch, 1, ss, 0, 1) == H.EINVAL
    assert H.hicr_channel_push(ch, 0, ss, N * T - T + 1, 1) == H.ERANGE
    assert H.hicr_channel_push(ch, 0, 99999, 0, 1) == H.EBADSLOT
    assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("P,E", [(4096 + 13, 8), (257, 3)])
def test_host_variable_spsc_lockstep(env, P, E):
    torch, H, wd, ctx = env
    seed = 57
    _say("host var spsc", P, E)
    g = np.random.default_rng(P)
    src_n = 1 << 16
    src = torch.empty(src_n, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), src_n, seed)
    ring = torch.zeros(P, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ss, rs, es = _reg(H, ctx, src), _reg(H, ctx, ring), _reg(H, ctx, ent)
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_HOST, rs, es,
                                                           capacity=P, entries=E))
    assert rc == H.OK
    oc = oracle.VChan(P, E)
    host_src = content(seed, 0, src_n)
    for step in range(600):
        if g.random() < 0.55:
            s = int(g.choice([0, 1, 15, 16, 17, P // 3, P // 2, P - 1, P, P + 1, int(g.integers(0, P))]))
            off = int(g.integers(0, src_n - s))
            rc = H.hicr_channel_push(ch, 0, ss, off, s)
            assert rc == oc.push(host_src[off:off + s], s)
            if rc == H.OK:
                assert H.hicr_fence(ctx) == H.OK
        else:
            n = int(g.integers(0, 3))
            m, b = oc.depth()
            assert H.hicr_channel_depth(ch, 0) == (H.OK, m, b)
            if m:
                dev_ring = ring.cpu().numpy()
                for i in range(min(n, m)):
                    rc, off, sz, _ = H.hicr_channel_peek(ch, 0, i)
                    ro, ooff, osz, _ = oc.peek(i)
                    assert (rc, off, sz) == (ro, ooff, osz)
                    got = np.concatenate([dev_ring[off:], dev_ring[:off]])[:sz]  # follows the wrap
                    assert np.array_equal(got, oc.read(i)[1])
            assert H.hicr_channel_pop(ch, 0, n) == oc.pop(n)
    assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_host_mpsc_lockstep(env, mode):
    torch, H, wd, ctx = env
    K, P, E, seed = 3, 2000, 4, 77
    _say("host mpsc", mode)
    g = np.random.default_rng(5)
    rings = 1 if mode == "lock" else K
    src_n = 1 << 15
    src = torch.empty(src_n, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), src_n, seed)
    ring = torch.zeros(rings * P, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(rings * E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ss, rs, es = _reg(H, ctx, src), _reg(H, ctx, ring), _reg(H, ctx, ent)
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, hmode, K, H.CH_HOST, rs, es,
                                                           capacity=P, entries=E))
    assert rc == H.OK, H.hicr_last_error(ctx)
    oc = oracle.MPSC(K, P, E, locking=(mode == "lock"))
    host_src = content(seed, 0, src_n)
    for step in range(500):
        if g.random() < 0.55:
            p = int(g.integers(0, K))
            s = int(g.integers(0, 900))
            off = int(g.integers(0, src_n - s))
            rc = H.hicr_channel_push(ch, p, ss, off, s)
            assert rc == oc.push(p, host_src[off:off + s], s)
            if rc == H.OK:
                assert H.hicr_fence(ctx) == H.OK
        else:
            r = int(g.integers(0, rings))
            oring = oc.rings[r]
            m, b = oring.depth()
            assert H.hicr_channel_depth(ch, r) == (H.OK, m, b)
            if m:
                dev = ring.cpu().numpy()[r * P:(r + 1) * P]
                rc, off, sz, prod = H.hicr_channel_peek(ch, r, 0)
                ro, ooff, osz, oprod = oring.peek(0)
                assert (rc, off - r * P, sz) == (ro, ooff, osz)
                assert prod == (oprod if mode == "lock" else r)
                local = off - r * P
                got = np.concatenate([dev[local:], dev[:local]])[:sz]
                assert np.array_equal(got, oring.read(0)[1])
            assert H.hicr_channel_pop(ch, r, 1) == oring.pop(1)
    assert H.hicr_channel_push(ch, K, ss, 0, 1) == H.EINVAL
    assert H.hicr_channel_destroy(ch) == H.OK


def test_channel_create_rejections(env):
    torch, H, wd, ctx = env
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    b = _reg(H, ctx, buf)
    small = _reg(H, ctx, buf, 0, 100)
    cfg = H.make_channel_cfg
    assert H.hicr_channel_create(ctx, cfg(H.CH_VAR, H.CH_SPSC, 2, H.CH_HOST, b, b, capacity=64,
                                          entries=4))[0] == H.EINVAL
    assert H.hicr_channel_create(ctx, cfg(H.CH_VAR, H.CH_MPSC_LOCK, 65, H.CH_HOST, b, b,
                                          capacity=64, entries=4))[0] == H.EINVAL
    assert H.hicr_channel_create(ctx, cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_HOST, small, b,
                                          capacity=101, entries=4))[0] == H.ERANGE
    assert H.hicr_channel_create(ctx, cfg(H.CH_FIXED, H.CH_SPSC, 1, H.CH_HOST, b, b,
                                          token_bytes=0, capacity=4))[0] == H.EINVAL
    assert H.hicr_channel_create(ctx, cfg(H.CH_VAR, H.CH_MPSC_NOLOCK, 4, H.CH_HOST, b, small,
                                          capacity=16, entries=4))[0] == H.ERANGE
    rc, dch = H.hicr_channel_create(ctx, cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_DEVICE, b, b,
                                             capacity=64, entries=4))
    assert rc == H.OK
    assert H.hicr_channel_push(dch, 0, b, 0, 1) == H.EINVAL     # device endpoints
    assert H.hicr_channel_destroy(dch) == H.OK


def test_pump_tiny_fixed_spsc(env):
    """The tiny channel driven by a producer wave and a consumer workgroup."""
    torch, H, wd, ctx = env
    C, T, N, seed = 16, 256, 1000, 91
    _say("pump tiny fixed")
    src = torch.empty(N * T, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), N * T, seed)
    out = torch.zeros(N * T, dtype=torch.uint8, device="cuda")
    ring = torch.zeros(C * T, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(C, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ss, os_, rs, es = _reg(H, ctx, src), _reg(H, ctx, out), _reg(H, ctx, ring), _reg(H, ctx, ent)
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_FIXED, H.CH_SPSC, 1, H.CH_DEVICE,
                                                           rs, es, token_bytes=T, capacity=C))
    assert rc == H.OK
    offs = np.arange(N, dtype=np.uint64) * T
    sizes = np.full(N, T, dtype=np.uint64)
    for rep in range(2):   # the channel is reusable: counters continue
        out.zero_()
        torch.cuda.synchronize()
        assert H.hicr_channel_pump(ctx, [(ch, 0, ss, os_, 0, N)], offs, sizes) == H.OK
        assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
        host_src = content(seed, 0, N * T)
        want = oracle_fifo_outputs(C * T, C, [host_src[i * T:(i + 1) * T] for i in range(N)])
        assert np.array_equal(out.cpu().numpy(), want)
    bad = sizes.copy()
    bad[5] = T - 1
    assert H.hicr_channel_pump(ctx, [(ch, 0, ss, os_, 0, N)], offs, bad) == H.EINVAL
    assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_pump_fixed_mpsc_and_spsc(env, mode):
    """Fixed-size channels through the pump: one MPSC channel of 4 producers
    and two SPSC channels, 256-byte tokens, 8-token rings, 400 tokens per
    stream read at scattered token-aligned offsets.  Every stream's output
    against the oracle (a locking channel's in the merge order its trace
    records, a non-locking one per producer)."""
    torch, H, wd, ctx = env
    C, T, N, K, seed = 8, 256, 400, 4, 97
    _say("pump fixed", mode)
    S = K + 2
    src_bytes = 2 * N * T
    src = torch.empty(S * src_bytes, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), S * src_bytes, seed)
    out = torch.zeros(S * N * T, dtype=torch.uint8, device="cuda")
    rings = K if mode == "nolock" else 1
    pay = torch.zeros((rings + 2) * C * T, dtype=torch.uint8, device="cuda")
    ent = torch.zeros((rings + 2) * C, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    chans = []
    r0 = 0
    for nr, m, k in ((rings, hmode, K), (1, H.CH_SPSC, 1), (1, H.CH_SPSC, 1)):
        ps = _reg(H, ctx, pay, r0 * C * T, nr * C * T)
        es = _reg(H, ctx, ent, r0 * C * 8, nr * C * 8)
        rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_FIXED, m, k, H.CH_DEVICE, ps,
                                                               es, token_bytes=T, capacity=C))
        assert rc == H.OK, H.hicr_last_error(ctx)
        chans.append(ch)
        r0 += nr
    g = np.random.default_rng(5)
    offs = (g.integers(0, src_bytes // T, S * N) * T).astype(np.uint64)
    sizes = np.full(S * N, T, dtype=np.uint64)
    streams = []
    for sidx in range(S):
        ch, p = (chans[0], sidx) if sidx < K else (chans[sidx - K + 1], 0)
        ss = _reg(H, ctx, src, sidx * src_bytes, src_bytes)
        os_ = _reg(H, ctx, out, sidx * N * T, N * T)
        streams.append((ch, p, ss, os_, sidx * N, N))
    trace = torch.zeros(S * N, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    assert H.hicr_channel_pump(ctx, streams, offs, sizes, trace.data_ptr(),
                               timeout_ns=5 * 10**9) == H.OK
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    host = content(seed, 0, S * src_bytes)
    msgs = [[host[sidx * src_bytes + int(o):sidx * src_bytes + int(o) + T]
             for o in offs[sidx * N:(sidx + 1) * N]] for sidx in range(S)]
    got = out.cpu().numpy().reshape(S, N * T)
    if mode == "lock":
        order = [int(x) for x in trace.cpu().numpy()[:K * N]]
        assert sorted(order) == sorted(list(range(K)) * N)
        want = oracle_locking_outputs(C * T, C, K, order, msgs[:K])
    else:
        want = [oracle_fifo_outputs(C * T, C, msgs[p]) for p in range(K)]
    for p in range(K):
        assert np.array_equal(got[p], want[p]), ("producer", p)
    for sidx in (K, K + 1):
        assert np.array_equal(got[sidx], oracle_fifo_outputs(C * T, C, msgs[sidx])), sidx
    for ch in chans:
        assert H.hicr_channel_destroy(ch) == H.OK


def _check_plan(torch, H, rig, plan, seed, mode, trace, sample=None):
    """Compare the pump's outputs with the oracle for every (or sampled)
    stream: each stream's whole output log, byte for byte, against the
    oracle's ring replayed with that stream's messages (a locking MPSC
    channel: its shared ring replayed in the device's consumption order)."""
    out = rig["out"]
    tr = trace.cpu().numpy() if trace is not None else None
    streams = list(range(plan.n_streams)) if sample is None else list(sample)
    want = expected_stream_outputs(plan, seed, mode, tr, streams)
    sb = plan.stream_bytes()

    def compare(sid):
        w = want[sid]
        assert len(w) == int(sb[sid]), ("stream length", sid)
        o = int(rig["out_off"][sid])
        got = out[o:o + len(w)].cpu().numpy()
        return bool(np.array_equal(got, w))

    ok = pmap(compare, sorted(want))
    bad = [sid for sid, k in zip(sorted(want), ok) if not k]
    assert not bad, ("streams differ from the oracle", bad[:8], len(bad))
    if tr is not None:
        # every channel's consumption order holds each of its streams n_msgs times
        per_chan = np.bincount(plan.stream_channel, weights=np.diff(plan.msg_begin),
                               minlength=plan.n_channels).astype(np.int64)
        base = np.concatenate([[0], np.cumsum(per_chan)[:-1]])
        for c in range(plan.n_channels):
            seg = tr[base[c]:base[c] + per_chan[c]]
            sids = [x for x in range(plan.n_streams) if plan.stream_channel[x] == c]
            cnt = np.bincount(seg, minlength=plan.n_streams)
            for sid in sids:
                assert cnt[sid] == plan.msg_begin[sid + 1] - plan.msg_begin[sid]
    return len(want)


@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_pump_small_mixed_plan(env, mode):
    """6 SPSC + 3 MPSC x 3 producers, small rings (8 KiB, 8 entries) so that
    producers wait for room and messages wrap; message sizes up to the ring."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 404
    _say("pump small", mode)
    plan = wc.plan(n_spsc=6, n_mpsc=3, K=3, total_msgs=1500, lo=1, hi=8192, P=8192, E=8,
                   src_bytes=1 << 16, batch=7)
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rig = channel_rig(torch, H, ctx, plan, hmode, seed)
    trace = torch.zeros(plan.n_msgs, dtype=torch.int32, device="cuda")
    ts = torch.zeros(2 * plan.n_msgs, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    rc = H.hicr_channel_pump(ctx, rig["streams"], plan.msg_src_off, plan.msg_size,
                             trace.data_ptr(), ts.data_ptr(), timeout_ns=5 * 10**9)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    _check_plan(torch, H, rig, plan, seed, mode, trace)
    t = ts.cpu().numpy().reshape(2, -1)
    assert (t[1] >= t[0]).all() and (t[0] > 0).all()
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK


def test_pumps_on_two_streams_sharing_channels_run_in_turn(env):
    """Every stream's messages split in two halves, pumped by two launches on
    two different streams with no fence between them: the second drives the
    same rings, so it must wait for the first (a ring has one producer and
    one consumer).  Each half writes its own output slot, placed so that the
    two halves of a stream make up its whole output log, which must equal the
    oracle's."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 405
    _say("pump two streams")
    plan = wc.plan(n_spsc=6, n_mpsc=3, K=3, total_msgs=1500, lo=1, hi=8192, P=8192, E=8,
                   src_bytes=1 << 16, batch=8)
    rig = channel_rig(torch, H, ctx, plan, H.CH_MPSC_NOLOCK, seed)
    out = rig["out"]
    halves = ([], [])
    for sid, (ch, p, ss, _os, first, n) in enumerate(rig["streams"]):
        h = n // 2
        b1 = int(plan.msg_size[first:first + h].sum())
        o = int(rig["out_off"][sid])
        for k, (f, m, base, size) in enumerate(((first, h, o, b1),
                                                (first + h, n - h, o + b1,
                                                 int(rig["stream_bytes"][sid]) - b1))):
            rc, slot = H.hicr_slot_register(ctx, out.data_ptr() + base, max(size, 1))
            assert rc == H.OK
            halves[k].append((ch, p, ss, slot, f, m))
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for k, st in enumerate((0, side.cuda_stream)):
        rc = H.hicr_channel_pump(ctx, halves[k], plan.msg_src_off, plan.msg_size,
                                 timeout_ns=5 * 10**9, stream=st)
        assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    assert _check_plan(torch, H, rig, plan, seed, "nolock", None) == plan.n_streams
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_pump_odd_ring_sizes(env, mode):
    """Rings of 8,191 bytes and 5 entries: messages (1..8,191 B) wrap at odd
    positions, so every wrap split starts and ends off the 16-byte grid."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 405
    _say("pump odd rings", mode)
    plan = wc.plan(n_spsc=5, n_mpsc=2, K=3, total_msgs=900, lo=1, hi=8191, P=8191, E=5,
                   src_bytes=1 << 16, batch=9)
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rig = channel_rig(torch, H, ctx, plan, hmode, seed)
    trace = torch.zeros(plan.n_msgs, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = H.hicr_channel_pump(ctx, rig["streams"], plan.msg_src_off, plan.msg_size,
                             trace.data_ptr(), 0, timeout_ns=5 * 10**9)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    _check_plan(torch, H, rig, plan, seed, mode, trace)
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("mode", ["lock", "nolock"])
@pytest.mark.parametrize("sizes", ["fixed", "mixed"])
def test_pump_held_batches_fill_the_ring(env, mode, sizes):
    """Streams of 320 messages, longer than four rings' worth of entries
    (E = 64), so the producers of rings of their own hold full batches of 16
    and publish up to 64 messages per release.  With 4 KiB messages through
    128 KiB rings two held batches fill a ring, so every third batch finds no
    room and has to publish the held ones before it waits; with sizes of
    1 B..8 KiB the ring fills at varying points.  The same bytes as the
    oracle, every stream whole."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 417
    _say("pump held batches", mode, sizes)
    lo, hi = (4096, 4096) if sizes == "fixed" else (1, 8192)
    plan = wc.plan(n_spsc=8, n_mpsc=2, K=3, total_msgs=14 * 320, lo=lo, hi=hi, P=32 * 4096,
                   E=64, src_bytes=1 << 20, batch=11)
    assert int(np.diff(plan.msg_begin).min()) > 4 * 64
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rig = channel_rig(torch, H, ctx, plan, hmode, seed)
    trace = torch.zeros(plan.n_msgs, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = H.hicr_channel_pump(ctx, rig["streams"], plan.msg_src_off, plan.msg_size,
                             trace.data_ptr(), 0, timeout_ns=5 * 10**9)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    _check_plan(torch, H, rig, plan, seed, mode, trace)
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_pump_device_tables(env, mode):
    """The small mixed plan with its message tables in device memory
    (HICR_PUMP_DEVICE_TABLES): the same bytes as the oracle, every message
    checked by its producer instead of the host."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 405
    _say("pump device tables", mode)
    plan = wc.plan(n_spsc=6, n_mpsc=3, K=3, total_msgs=1500, lo=1, hi=8192, P=8192, E=8,
                   src_bytes=1 << 16, batch=7)
    plan.msg_size[::37] = 0  # zero-byte messages take an entry and no bytes
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rig = channel_rig(torch, H, ctx, plan, hmode, seed)
    trace = torch.zeros(plan.n_msgs, dtype=torch.int32, device="cuda")
    offs = torch.from_numpy(plan.msg_src_off.astype(np.int64)).cuda()
    sizes = torch.from_numpy(plan.msg_size.astype(np.int64)).cuda()
    torch.cuda.synchronize()
    rc = H.hicr_channel_pump(ctx, rig["streams"], offs.data_ptr(), sizes.data_ptr(),
                             trace.data_ptr(), timeout_ns=5 * 10**9, n_msgs=plan.n_msgs)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    _check_plan(torch, H, rig, plan, seed, mode, trace)
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK


@pytest.mark.parametrize("bad", ["size", "offset"])
def test_pump_device_tables_bad_message_is_reported(env, bad):
    """A message in device tables that does not fit its ring (or lies outside
    its source slot) is caught by its producer before a byte moves: the pump
    ends, the fence reports HICR_EDEVICE and the channel is broken.  Fixed-size
    channels and unknown flags are refused on the host."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    _say("pump device tables bad", bad)
    plan = wc.plan(n_spsc=4, n_mpsc=0, K=1, total_msgs=200, lo=1, hi=4096, P=8192, E=8,
                   src_bytes=1 << 16, batch=7)
    rig = channel_rig(torch, H, ctx, plan, H.CH_MPSC_NOLOCK, 11)
    o = plan.msg_src_off.astype(np.int64).copy()
    z = plan.msg_size.astype(np.int64).copy()
    k = int(plan.msg_begin[2]) + 5  # a message of stream 2
    if bad == "size":
        z[k] = plan.P + 1
    else:
        o[k] = plan.src_bytes - int(z[k]) + 1
    offs, sizes = torch.from_numpy(o).cuda(), torch.from_numpy(z).cuda()
    torch.cuda.synchronize()
    rc = H.hicr_channel_pump(ctx, rig["streams"], offs.data_ptr(), sizes.data_ptr(),
                             timeout_ns=2 * 10**9, n_msgs=plan.n_msgs)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.EDEVICE
    # the channel the bad message went through is broken
    assert H.hicr_channel_pump(ctx, rig["streams"], plan.msg_src_off, plan.msg_size) == H.EINVAL
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK
    # unknown flag bits are refused before anything runs
    io = H.hicr_pump_io(None, None, 0, None, None, 0, 0x2, 0)
    arr = (H.hicr_stream * 1)()
    assert H.lib().hicr_channel_pump(ctx, arr, 0, H.ctypes.byref(io), None) == H.EINVAL


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["lock", "nolock"])
def test_pump_full_size_every_stream(env, mode):
    """The measured channel configuration in the benchmark's launch: 1,024
    SPSC + 64 MPSC x 8 producers, 1e6 messages of 16 B..256 KiB through 1 MiB
    / 64-entry rings, message tables resident on the device, one persistent
    launch.  Every one of the 1,536 streams' output logs is compared whole
    with the oracle (locking channels: replayed in the device's consumption
    order, which must merge the producers' sequences); every channel's
    consumption order holds each of its streams' messages."""
    torch, H, wd, ctx = env
    from bench import channel_rig
    seed = 808
    _say("pump full", mode)
    plan = wc.plan()
    hmode = H.CH_MPSC_LOCK if mode == "lock" else H.CH_MPSC_NOLOCK
    rig = channel_rig(torch, H, ctx, plan, hmode, seed)
    trace = torch.zeros(plan.n_msgs, dtype=torch.int32, device="cuda")
    ts = torch.zeros(2 * plan.n_msgs, dtype=torch.int64, device="cuda")
    offs = torch.from_numpy(plan.msg_src_off.astype(np.int64)).cuda()
    sizes = torch.from_numpy(plan.msg_size.astype(np.int64)).cuda()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rc = H.hicr_channel_pump(ctx, rig["streams"], offs.data_ptr(), sizes.data_ptr(),
                             trace.data_ptr(), ts.data_ptr(), timeout_ns=10 * 10**9,
                             n_msgs=plan.n_msgs)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    payload = int(plan.msg_size.sum())
    t = ts.cpu().numpy().reshape(2, -1).astype(np.int64)
    lat_us = (t[1] - t[0]) / 100.0
    _say(f"pump {mode}: {ms:.2f} ms, {4 * payload / ms / 1e6:.0f} GB/s (4 x payload), "
         f"latency p50 {np.percentile(lat_us, 50):.1f} us p99 {np.percentile(lat_us, 99):.1f} us")
    n = _check_plan(torch, H, rig, plan, seed, mode, trace)
    assert n == plan.n_streams == 1536
    _say(f"pump {mode}: all {n} streams equal the oracle")
    for ch in rig["channels"]:
        assert H.hicr_channel_destroy(ch) == H.OK
    del rig
    torch.cuda.empty_cache()


def _blocking_rig(torch, H, wd, ctx, n_msgs, msg_bytes, P, E, locking=False):
    """A device channel whose ring is far smaller than the traffic, so that
    producers must wait for room again and again."""
    src = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), 1 << 20, 3)
    out = torch.zeros(n_msgs * msg_bytes + 64, dtype=torch.uint8, device="cuda")
    ring = torch.zeros(P, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    ss, os_, rs, es = _reg(H, ctx, src), _reg(H, ctx, out), _reg(H, ctx, ring), _reg(H, ctx, ent)
    mode = H.CH_MPSC_LOCK if locking else H.CH_SPSC
    K = 2 if locking else 1
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, mode, K, H.CH_DEVICE, rs, es,
                                                           capacity=P, entries=E))
    assert rc == H.OK, H.hicr_last_error(ctx)
    g = np.random.default_rng(n_msgs)
    offs = (g.random(n_msgs) * ((1 << 20) - msg_bytes)).astype(np.uint64)
    sizes = np.full(n_msgs, msg_bytes, dtype=np.uint64)
    streams = [(ch, 0, ss, os_, 0, n_msgs)]
    return ch, streams, offs, sizes, (src, out, ring, ent)


@pytest.mark.parametrize("locking", [False, True])
def test_pump_timeout_is_reported_and_breaks_the_channel(env, locking):
    """A no-progress limit of one device-clock tick ends the pump at its
    first wait: every wave exits, the fence reports HICR_ETIMEDOUT, the
    channel refuses further pumps, and the context keeps working."""
    torch, H, wd, ctx = env
    _say("pump timeout", locking)
    ch, streams, offs, sizes, keep = _blocking_rig(torch, H, wd, ctx, 2000, 4096, 8192, 4, locking)
    assert H.hicr_channel_pump(ctx, streams, offs, sizes, timeout_ns=1) == H.OK
    assert H.hicr_fence(ctx) == H.ETIMEDOUT
    assert H.hicr_channel_pump(ctx, streams, offs, sizes) == H.EINVAL
    assert H.hicr_fence(ctx) == H.OK
    # the context still moves bytes
    a = torch.arange(256, dtype=torch.uint8, device="cuda")
    b = torch.zeros(256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    sa, sb = _reg(H, ctx, a), _reg(H, ctx, b)
    assert H.hicr_memcpy(ctx, sb, 0, sa, 0, 256) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    assert np.array_equal(b.cpu().numpy(), np.arange(256, dtype=np.uint8))
    assert H.hicr_channel_destroy(ch) == H.OK


def test_pump_abort_ends_a_running_pump(env):
    """hicr_channel_abort while a long pump runs (60,000 messages through an
    8 KiB ring): the pump ends early and the fence reports the abort."""
    import time
    torch, H, wd, ctx = env
    _say("pump abort")
    ch, streams, offs, sizes, keep = _blocking_rig(torch, H, wd, ctx, 60000, 4096, 8192, 4)
    t0 = time.perf_counter()
    assert H.hicr_channel_pump(ctx, streams, offs, sizes, timeout_ns=5 * 10**9) == H.OK
    time.sleep(0.002)
    assert H.hicr_channel_abort(ctx) == H.OK
    rc = H.hicr_fence(ctx)
    dt = time.perf_counter() - t0
    assert rc == H.EDEVICE, (rc, H.hicr_last_error(ctx), dt)
    assert "abort" in H.hicr_last_error(ctx)
    assert H.hicr_channel_pump(ctx, streams, offs, sizes) == H.EINVAL
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_channel_destroy(ch) == H.OK


def test_pump_abort_reaches_a_pump_that_shares_its_queue(env):
    """hicr_channel_abort is a store into the pump's pinned abort word, so it
    reaches a running pump whatever hardware queue the pump's stream shares:
    the pump runs on one of twelve streams that all have had work (more
    streams than the process's hardware queues), and ends early with the
    abort reported."""
    import time
    torch, H, wd, ctx = env
    _say("pump abort, twelve busy streams")
    streams_t = [torch.cuda.Stream() for _ in range(12)]
    busy = []
    for st_ in streams_t:
        with torch.cuda.stream(st_):
            x = torch.zeros(1 << 16, device="cuda")
            x += 1
            busy.append(x)
    torch.cuda.synchronize()
    ch, streams, offs, sizes, keep = _blocking_rig(torch, H, wd, ctx, 60000, 4096, 8192, 4)
    t0 = time.perf_counter()
    assert H.hicr_channel_pump(ctx, streams, offs, sizes, timeout_ns=5 * 10**9,
                               stream=streams_t[7].cuda_stream) == H.OK
    time.sleep(0.002)
    assert H.hicr_channel_abort(ctx) == H.OK
    rc = H.hicr_fence(ctx)
    dt = time.perf_counter() - t0
    assert rc == H.EDEVICE, (rc, H.hicr_last_error(ctx), dt)
    assert "abort" in H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_channel_destroy(ch) == H.OK
    torch.cuda.synchronize()
