"""Helpers that turn oracle results into expected device contents.

Expected values come only from the CPU oracle (``oracle``) applied to inputs
drawn by ``workloads``; nothing here reads the GPU library's results except
the arrays handed in for comparison.
"""
import concurrent.futures as cf
import os

import numpy as np

import oracle
from workloads.content import content


def workers() -> int:
    """Host threads for whole-output checks (numpy and the oracle's C code
    release the interpreter lock); at most 16, the share of one GPU's host."""
    return max(1, min(16, os.cpu_count() or 1))


def pmap(fn, items):
    """fn over items on a thread pool, results in order."""
    with cf.ThreadPoolExecutor(max_workers=workers()) as ex:
        return list(ex.map(fn, items))


def abs_ranges(descs, bases):
    """Absolute (dst, src, size) of every request given slot base offsets."""
    dabs = np.asarray(bases, dtype=np.uint64)[descs["dst_slot"]] + descs["dst_off"]
    sabs = np.asarray(bases, dtype=np.uint64)[descs["src_slot"]] + descs["src_off"]
    return dabs.astype(np.int64), sabs.astype(np.int64), descs["size"].astype(np.int64)


def expected_window(dabs, sabs, size, w0, w1, seed):
    """Bytes [w0, w1) of a pool filled under ``seed`` after one hazard-free
    batch: the oracle's memcpy applied, in index order, to every request whose
    destination meets the window (clipped to it), each reading its source from
    the content as it was at the start of the epoch."""
    win = content(seed, w0, w1 - w0)
    c = oracle.Ctx()
    rc, wslot = c.register(win)
    assert rc == oracle.OK
    hit = np.nonzero((dabs < w1) & (dabs + size > w0) & (size > 0))[0]
    for j in hit:
        x0 = max(int(dabs[j]), w0)
        x1 = min(int(dabs[j] + size[j]), w1)
        src = content(seed, int(sabs[j]) + (x0 - int(dabs[j])), x1 - x0)
        rc, sslot = c.register(src)
        assert rc == oracle.OK
        assert c.memcpy(wslot, x0 - w0, sslot, 0, x1 - x0) == oracle.OK
    return win


def oracle_counters(descs, n_slots):
    """Per-slot (sent, recv) after one batch, from the oracle's counter rule."""
    c = oracle.Ctx()
    dummy = np.zeros(1, np.uint8)
    # Slots of size 2^62 at one shared address: only the counter effect is
    # used (count_batch moves no bytes), so bounds never bind.
    for _ in range(n_slots):
        rc, _s = c.register_raw(dummy.ctypes.data, 1 << 62)
        assert rc == oracle.OK
    rc, bad = c.count_batch(descs)
    assert rc == oracle.OK, (rc, bad)
    out = np.zeros((n_slots, 2), dtype=np.uint64)
    for k in range(n_slots):
        _, s, r = c.counters(k)
        out[k] = (s, r)
    return out


def oracle_fifo_outputs(P, E, stream_msgs):
    """Consumer output of one SPSC (or non-locking MPSC sub-) ring: the
    oracle's variable ring driven by a sequential schedule (push while there
    is room, otherwise read and pop the oldest), so the output is the order
    the oracle's FIFO defines.  stream_msgs: list of uint8 arrays."""
    ch = oracle.VChan(P, E)
    out = []
    for m in stream_msgs:
        while True:
            rc = ch.push(m, len(m))
            if rc == oracle.OK:
                break
            assert rc == oracle.EAGAIN
            rc, data, _ = ch.read(0)
            out.append(data)
            assert ch.pop(1) == oracle.OK
    while ch.depth()[0]:
        rc, data, _ = ch.read(0)
        out.append(data)
        assert ch.pop(1) == oracle.OK
    return np.concatenate(out) if out else np.zeros(0, np.uint8)


def oracle_locking_outputs(P, E, K, order, stream_msgs_by_prod):
    """Outputs of a locking MPSC channel whose consumer took producers'
    messages in ``order`` (list of producer ids): the oracle's shared tagged
    ring replays that merge; the consumer routes by the entry's producer."""
    ch = oracle.MPSC(K, P, E, locking=True)
    nxt = [0] * K
    outs = [[] for _ in range(K)]
    ring = ch.ring_for(0)
    for p in order:
        m = stream_msgs_by_prod[p][nxt[p]]
        nxt[p] += 1
        while True:
            rc = ch.push(p, m, len(m))
            if rc == oracle.OK:
                break
            assert rc == oracle.EAGAIN
            rc, data, prod = ring.read(0)
            outs[prod].append(data)
            assert ring.pop(1) == oracle.OK
    while ring.depth()[0]:
        rc, data, prod = ring.read(0)
        outs[prod].append(data)
        assert ring.pop(1) == oracle.OK
    assert nxt == [len(x) for x in stream_msgs_by_prod], "trace is not a merge of the streams"
    return [np.concatenate(o) if o else np.zeros(0, np.uint8) for o in outs]


def stream_blob_msgs(plan, seed, s):
    """Source bytes of stream s (its whole source slot) and the (offset,
    size) of each of its messages inside them."""
    b0, b1 = int(plan.msg_begin[s]), int(plan.msg_begin[s + 1])
    blob = content(seed, s * plan.src_bytes, plan.src_bytes)
    return blob, plan.msg_src_off[b0:b1], plan.msg_size[b0:b1]


def expected_stream_outputs(plan, seed, mode, trace, streams):
    """Oracle output of every stream in ``streams`` (stream id -> bytes).
    A ring with one producer (an SPSC channel, or a non-locking MPSC
    sub-ring) is replayed through the oracle's ring alone; a locking MPSC
    channel's shared ring is replayed in the order the device consumed its
    producers' messages (``trace``: stream id per consumed message, channels
    in stream order), which must be a merge of their sequences."""
    per_chan = np.bincount(plan.stream_channel, weights=np.diff(plan.msg_begin),
                           minlength=plan.n_channels).astype(np.int64)
    base = np.concatenate([[0], np.cumsum(per_chan)[:-1]])
    jobs, seen = [], set()
    for s in streams:
        c = int(plan.stream_channel[s])
        if c < plan.n_spsc or mode == "nolock":
            jobs.append(("one", s))
        elif c not in seen:
            seen.add(c)
            jobs.append(("lock", c))

    def run(job):
        kind, x = job
        if kind == "one":
            blob, o, z = stream_blob_msgs(plan, seed, x)
            rc, outs = oracle.vchan_replay(plan.P, plan.E, np.zeros(len(z), np.uint32),
                                           [blob], [o], [z])
            assert rc == oracle.OK, ("replay", x, rc)
            return {x: outs[0]}
        sids = [q for q in range(plan.n_streams) if plan.stream_channel[q] == x]
        prod_of = {q: int(plan.stream_producer[q]) for q in sids}
        by_prod = [None] * plan.K
        for q in sids:
            by_prod[prod_of[q]] = stream_blob_msgs(plan, seed, q)
        order = np.array([prod_of[int(q)] for q in trace[base[x]:base[x] + per_chan[x]]],
                         dtype=np.uint32)
        rc, outs = oracle.vchan_replay(plan.P, plan.E, order, [b[0] for b in by_prod],
                                       [b[1] for b in by_prod], [b[2] for b in by_prod],
                                       tagged=True)
        assert rc == oracle.OK, ("locking replay: not a merge of the streams", x, rc)
        return {q: outs[prod_of[q]] for q in sids}

    out = {}
    for r in pmap(run, jobs):
        out.update(r)
    return out
