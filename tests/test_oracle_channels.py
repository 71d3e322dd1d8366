"""Pins of the oracle's channels (CPU only).

Independent models the oracle is checked against:
  * a Python ``deque`` of messages with a byte/entry budget -- the textbook
    bounded FIFO queue (Lamport's single-producer single-consumer ring with
    monotone counters behaves exactly like it);
  * exhaustive enumeration of every push/pop attempt sequence up to a depth;
  * closed forms: a one-token channel forces strict push/pop alternation (the
    paper's ping-pong benchmark uses a single-message buffer for exactly this);
    fixed-size rings equal variable-size rings whose messages all have T bytes;
  * the step-level protocol explorer, which must accept the protocol and
    reject every planted mistake.
"""
import itertools
from collections import deque

import numpy as np
import pytest

from oracle import protocol
from workloads import channels as wc
from workloads.content import content


class QueueModel:
    """Bounded FIFO of messages: entries <= E and bytes <= P."""

    def __init__(self, P, E):
        self.P, self.E = P, E
        self.q = deque()
        self.bytes = 0

    def push(self, msg):
        if len(msg) > self.P:
            return -1
        if len(self.q) == self.E or self.bytes + len(msg) > self.P:
            return -5
        self.q.append(msg)
        self.bytes += len(msg)
        return 0

    def pop(self, n):
        if n > len(self.q):
            return -5
        for _ in range(n):
            self.bytes -= len(self.q.popleft())
        return 0


def test_fixed_spsc_tiny_schedule(orc):
    """The tiny channel (16 tokens x 256 B, 1,000 tokens) driven by the seeded
    attempt schedule, against the queue model, token by token."""
    C, T, N = 16, 256, 1000
    ch = orc.FChan(C, T)
    model = QueueModel(C * T, C)
    src = content(21, 0, N * T)
    sent = popped = 0
    out = []
    for kind, k in wc.tiny_schedule() + [("pop", 1)] * (2 * N):
        if popped == N:
            break
        if kind == "push":
            k = min(k, N - sent)
            if k == 0:
                continue
            rc = ch.push(src[sent * T:], k)
            toks = [src[(sent + t) * T:(sent + t + 1) * T].tobytes() for t in range(k)]
            want = 0 if C - len(model.q) >= k else -5
            if want == 0:
                for tk in toks:
                    model.push(tk)
            assert rc == want
            if rc == 0:
                sent += k
        else:
            for i in range(min(k, ch.depth())):
                rc, off = ch.peek(i)
                assert rc == 0
                assert ch.ring[off:off + T].tobytes() == model.q[i]
            rc = ch.pop(k)
            assert rc == model.pop(k)
            if rc == 0:
                out += [None] * k
                popped += k
        assert 0 <= ch.tail - ch.head <= C
        assert ch.depth() == len(model.q)
    assert popped == N and sent == N


def test_fixed_one_token_alternates(orc):
    ch = orc.FChan(1, 8)
    a = np.arange(8, dtype=np.uint8)
    for _ in range(20):
        assert ch.push(a, 1) == 0
        assert ch.push(a, 1) == orc.EAGAIN       # full: wait for the consumer
        assert ch.peek(0) == (0, 0)
        assert ch.pop(1) == 0
        assert ch.pop(1) == orc.EAGAIN           # empty
        assert ch.peek(0)[0] == orc.EAGAIN


def test_fixed_rejects_and_all_or_nothing(orc):
    assert orc.FChan(0, 8).rc_init == orc.EINVAL
    assert orc.FChan(4, 0).rc_init == orc.EINVAL
    ch = orc.FChan(3, 2)       # capacity not a power of two
    a = np.arange(20, dtype=np.uint8)
    assert ch.push(a, 4) == orc.EINVAL          # can never fit
    assert ch.push(a, 2) == 0
    assert ch.push(a[4:], 2) == orc.EAGAIN      # one free token, asked for two
    assert ch.depth() == 2 and ch.tail == 2
    assert ch.pop(1) == 0
    assert ch.push(a[4:], 2) == 0               # wraps: tokens land in slots 2 then 0
    assert list(ch.ring) == [6, 7, 2, 3, 4, 5]
    assert [ch.peek(i)[1] for i in range(3)] == [2, 4, 0]


def test_fixed_equals_variable_with_constant_size(orc):
    g = np.random.default_rng(5)
    C, T = 5, 3
    f = orc.FChan(C, T)
    v = orc.VChan(C * T, C)
    src = g.integers(0, 256, 3000, dtype=np.uint8)
    pos = 0
    for _ in range(600):
        if g.random() < 0.55:
            rf = f.push(src[pos:], 1)
            rv = v.push(src[pos:], T)
            assert rf == rv
            pos += T if rf == 0 else 0
        else:
            assert f.pop(1) == v.pop(1)
        assert f.depth() == v.depth()[0]
        for i in range(f.depth()):
            assert f.peek(i)[1] == v.peek(i)[1]


def test_variable_spsc_against_queue(orc):
    g = np.random.default_rng(9)
    for P, E in [(16, 4), (17, 3), (64, 64), (5, 1), (1, 2)]:
        v = orc.VChan(P, E)
        m = QueueModel(P, E)
        for step in range(3000):
            if g.random() < 0.5:
                s = int(g.integers(0, P + 3))
                msg = g.integers(0, 256, max(s, 1), dtype=np.uint8)[:s]
                rc = v.push(msg, s)
                assert rc == m.push(msg.tobytes())
            else:
                n = int(g.integers(0, 3))
                assert v.pop(n) == m.pop(n)
            msgs, nbytes = v.depth()
            assert msgs == len(m.q) and nbytes == m.bytes
            hm, tm, hb, tb = v.state
            assert 0 <= tm - hm <= E and 0 <= tb - hb <= P
            # every message reads back intact and sits right after the last
            off = hb % P
            for i in range(msgs):
                rc, o, s, _ = v.peek(i)
                assert rc == 0 and o == off and s == len(m.q[i])
                assert v.read(i)[1].tobytes() == m.q[i]
                off = (off + s) % P


def test_variable_zero_and_full_size_messages(orc):
    v = orc.VChan(8, 3)
    assert v.push(np.zeros(0, np.uint8), 0) == 0           # zero-byte message uses an entry
    assert v.push(np.arange(8, dtype=np.uint8), 8) == 0    # exactly the ring
    assert v.push(np.zeros(0, np.uint8), 0) == 0
    assert v.push(np.zeros(0, np.uint8), 0) == orc.EAGAIN  # entries exhausted
    assert v.push(np.zeros(9, np.uint8), 9) == orc.EINVAL  # larger than the ring
    assert v.depth() == (3, 8)
    assert v.pop(2) == 0
    assert v.push(np.arange(10, 15, dtype=np.uint8), 5) == 0
    # the 5-byte message started at byte 0 again (8 mod 8) -- no split
    assert v.peek(1)[1:3] == (0, 5)
    assert v.pop(1) == 0
    assert v.push(np.arange(20, 23, dtype=np.uint8), 3) == 0   # lands at 5,6,7
    assert v.push(np.zeros(1, np.uint8), 1) == orc.EAGAIN      # ring holds 8 bytes
    assert list(v.payload) == [10, 11, 12, 13, 14, 20, 21, 22]
    assert v.pop(1) == 0
    assert v.push(np.arange(30, 34, dtype=np.uint8), 4) == 0   # wraps across the end? no: 0..3
    assert v.read(1)[1].tolist() == [30, 31, 32, 33]
    # force a split: drain, then offset the tail to 6 and push 4 bytes
    v2 = orc.VChan(8, 4)
    assert v2.push(np.zeros(6, np.uint8), 6) == 0 and v2.pop(1) == 0
    assert v2.push(np.arange(1, 5, dtype=np.uint8), 4) == 0
    assert list(v2.payload[6:]) == [1, 2] and list(v2.payload[:2]) == [3, 4]
    assert v2.read(0)[1].tolist() == [1, 2, 3, 4]


def test_operation_level_exhaustive(orc):
    """Every sequence of attempts up to depth 8 over a tiny ring, each push
    offering the next message of a fixed list; compared to the queue model
    after every step."""
    sizes = [2, 0, 3, 1, 4, 2]
    P, E = 5, 3
    msgs = [bytes(range(10 * i, 10 * i + s)) for i, s in enumerate(sizes)]
    n_seq = 0
    for depth in range(1, 9):
        for seq in itertools.product([0, 1, 2], repeat=depth):  # 0 push, 1 pop1, 2 pop2
            v = orc.VChan(P, E)
            m = QueueModel(P, E)
            nxt = 0
            for a in seq:
                if a == 0:
                    if nxt == len(msgs):
                        continue
                    arr = np.frombuffer(msgs[nxt], np.uint8).copy()
                    rc = v.push(arr, len(arr))
                    assert rc == m.push(msgs[nxt])
                    nxt += rc == 0
                else:
                    assert v.pop(a) == m.pop(a)
                assert v.depth() == (len(m.q), m.bytes)
                for i in range(len(m.q)):
                    assert v.read(i)[1].tobytes() == m.q[i]
            n_seq += 1
    assert n_seq == sum(3 ** d for d in range(1, 9))


@pytest.mark.parametrize("locking", [True, False])
def test_mpsc_fifo_per_producer_and_merge(orc, locking):
    g = np.random.default_rng(11 + locking)
    K = 3
    ch = orc.MPSC(K, 32, 4, locking)
    pending = [deque(g.integers(0, 256, int(g.integers(0, 9)), dtype=np.uint8).tobytes()
                     for _ in range(20)) for _ in range(K)]
    pushed = [[] for _ in range(K)]
    got = [[] for _ in range(K)]
    order = []
    while any(pending) or any(r.depth()[0] for r in ch.rings):
        if g.random() < 0.6 and any(pending):
            p = int(g.choice([k for k in range(K) if pending[k]]))
            msg = pending[p][0]
            rc = ch.push(p, np.frombuffer(msg, np.uint8).copy(), len(msg))
            if rc == 0:
                pushed[p].append(pending[p].popleft())
            else:
                assert rc == orc.EAGAIN
        else:
            rings = [r for r in range(len(ch.rings)) if ch.rings[r].depth()[0]]
            if not rings:
                continue
            r = ch.rings[int(g.choice(rings))]
            rc, data, prod = r.read(0)
            prod = prod if locking else ch.rings.index(r)
            got[prod].append(data.tobytes())
            order.append(prod)
            assert r.pop(1) == 0
    assert got == pushed                      # per-producer FIFO, nothing lost
    assert sorted(order) == sorted(p for p in range(K) for _ in pushed[p])
    assert ch.push(K, np.zeros(1, np.uint8), 1) == orc.EINVAL


# --------------------------------------------------- step-level protocol

CASES = [
    (4, 2, [[1, 2, 3]], False),          # SPSC, wraps, entry limit 2
    (3, 1, [[3, 0, 2]], False),          # one entry: strict alternation
    (5, 3, [[2, 5, 1]], False),          # a message as large as the ring
    (4, 2, [[2, 1], [1, 2]], True),      # locking MPSC
    (3, 2, [[1, 2], [2, 1]], False),     # non-locking MPSC
]


@pytest.mark.parametrize("P,E,msgs,locking", CASES)
def test_protocol_explorer_accepts(P, E, msgs, locking):
    n = protocol.explore(P, E, msgs, locking=locking)
    assert n > 20


@pytest.mark.parametrize("bug", ["publish_before_payload", "free_before_read",
                                 "room_off_by_one"])
def test_protocol_explorer_catches_planted_bugs(bug):
    v = protocol.Variant(**{bug: True})
    with pytest.raises(protocol.Violation):
        protocol.explore(4, 2, [[1, 3, 2]], variant=v)


def test_protocol_explorer_catches_missing_lock():
    with pytest.raises(protocol.Violation):
        protocol.explore(4, 2, [[2, 1], [1, 2]], locking=True,
                         variant=protocol.Variant(no_lock=True))


def test_channel_plan_shape():
    p = wc.plan()
    assert p.n_streams == 1536 and p.n_msgs == 1_000_000
    per = np.diff(p.msg_begin)
    assert (per[:64] == 652).all() and (per[64:] == 651).all()
    assert (p.msg_size >= 16).all() and (p.msg_size <= 256 * 1024).all()
    assert (p.msg_src_off + p.msg_size <= p.src_bytes).all()
    assert 25e9 < int(p.msg_size.sum()) < 29e9           # ~27.0 GB of payload
    assert (np.bincount(p.stream_channel) == np.r_[np.ones(1024), 8 * np.ones(64)]).all()


@pytest.mark.parametrize("P,E,msgs", [(4, 2, [[2, 1], [1, 2]]), (5, 3, [[2, 1], [1, 2], [3]]),
                                      (3, 1, [[1, 1], [2]])])
def test_protocol_reservation_locking_accepts(P, E, msgs):
    """Locking MPSC that holds the lock only for the room check and the
    reservation, copies outside it and publishes in lock order."""
    assert protocol.explore(P, E, msgs, locking=True, reserve=True) > 50


def test_protocol_reservation_catches_unordered_publish_and_no_lock():
    with pytest.raises(protocol.Violation):
        protocol.explore(4, 3, [[2, 1], [1, 2]], locking=True, reserve=True,
                         variant=protocol.Variant(unordered_publish=True))
    with pytest.raises(protocol.Violation):
        protocol.explore(4, 2, [[2, 1], [1, 2]], locking=True, reserve=True,
                         variant=protocol.Variant(no_lock=True))


# ------------------------------------------- whole-ring replay (test harness)

def test_replay_spsc_output_is_the_fifo_concatenation(orc):
    """or_vchan_replay on one producer: whatever the ring's size, entry
    count, wraps and back-pressure, the consumer's output is every message in
    push order (the FIFO definition), byte for byte."""
    g = np.random.default_rng(31)
    for case in range(300):
        P = int(g.integers(1, 65))
        E = int(g.integers(1, 9))
        n = int(g.integers(0, 40))
        blob = g.integers(0, 256, 4096, dtype=np.uint8)
        sizes = g.integers(0, P + 1, n).astype(np.uint64)
        offs = np.array([g.integers(0, 4096 - int(z) + 1) for z in sizes], dtype=np.uint64)
        rc, outs = orc.vchan_replay(P, E, np.zeros(n, np.uint32), [blob], [offs], [sizes])
        assert rc == orc.OK, case
        want = np.concatenate([blob[int(o):int(o) + int(z)] for o, z in zip(offs, sizes)]
                              + [np.zeros(0, np.uint8)])
        assert np.array_equal(outs[0], want), case


def test_replay_tagged_routes_each_producer_in_its_order(orc):
    """Tagged (locking MPSC) replay of a random merge of three producers'
    sequences: producer p's output is its own messages in its own order."""
    g = np.random.default_rng(32)
    for case in range(100):
        K, P, E = 3, int(g.integers(8, 65)), int(g.integers(1, 6))
        blobs = [g.integers(0, 256, 1024, dtype=np.uint8) for _ in range(K)]
        sizes = [g.integers(0, P + 1, int(g.integers(0, 12))).astype(np.uint64) for _ in range(K)]
        offs = [np.array([g.integers(0, 1024 - int(z) + 1) for z in zp], dtype=np.uint64)
                for zp in sizes]
        order = np.concatenate([np.full(len(z), p, np.uint32) for p, z in enumerate(sizes)])
        g.shuffle(order)
        rc, outs = orc.vchan_replay(P, E, order, blobs, offs, sizes, tagged=True)
        assert rc == orc.OK, case
        for p in range(K):
            want = np.concatenate([blobs[p][int(o):int(o) + int(z)]
                                   for o, z in zip(offs[p], sizes[p])] + [np.zeros(0, np.uint8)])
            assert np.array_equal(outs[p], want), (case, p)


def test_replay_rejects_bad_schedules(orc):
    blob = np.arange(64, dtype=np.uint8)
    one = [np.array([0], np.uint64)], [np.array([4], np.uint64)]
    # a producer named more often than it has messages
    assert orc.vchan_replay(8, 2, [0, 0], [blob], *one)[0] == orc.EINVAL
    # an unknown producer
    assert orc.vchan_replay(8, 2, [1], [blob], *one)[0] == orc.EINVAL
    # a message larger than the ring
    assert orc.vchan_replay(3, 2, [0], [blob], *one)[0] == orc.EINVAL
    with pytest.raises(ValueError):
        orc.vchan_replay(8, 2, [0], [blob], [np.array([62], np.uint64)], [np.array([4], np.uint64)])
